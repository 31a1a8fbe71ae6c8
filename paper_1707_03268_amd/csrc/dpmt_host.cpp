// Host runtime of libdpmt: context, validation, FP64 decomposition of the
// filter bank, operand packing, planning of work lists, and the launch
// sequence of dpmt_score_pyramid.  Kernels live in dpmt_kernels.hip.
#include "dpmt.h"
#include "dpmt_hog.h"
#include "dpmt_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

using namespace dpmt;

namespace {

thread_local std::string g_free_error;   // errors of calls without a context

// Correlation tile configurations the autotuner chooses from: output rows per
// wave, 32-filter blocks per wave, waves per workgroup, resident grid, groups
// of filter blocks walked over one window, and how many of the waves sit side
// by side along x (the rest stacked along rows).  All of them accumulate
// every response in the same order, so they give equal bits.  Wider
// workgroup tiles write longer runs of every response row: the FP32
// responses leave in 128-byte runs per filter row with one wave along x, in
// 512- or 1024-byte runs with 4 or 8.
struct TileCfg {
    int ty, bb, wy, persistent;
    int nfb;           // groups of bb filter blocks a tile walks over one window
    const char* name;
    int wx;            // waves along x
};
constexpr TileCfg TILE_CFGS[] = {
    {4, 2, 4, 0, 1, "16 rows x 32 cols x 64 filters, 256 threads, one workgroup per tile", 1},
    {4, 2, 4, 1, 1, "16 rows x 32 cols x 64 filters, 256 threads, resident grid", 1},
    {2, 2, 4, 0, 1, "8 rows x 32 cols x 64 filters, 256 threads, one workgroup per tile", 1},
    {4, 1, 4, 0, 1, "16 rows x 32 cols x 32 filters, 256 threads, one workgroup per tile", 1},
    {2, 2, 4, 1, 1, "8 rows x 32 cols x 64 filters, 256 threads, resident grid", 1},
    {4, 1, 4, 0, 6, "16 rows x 32 cols x 6 x 32 filters over one window, 256 threads", 1},
    {4, 1, 4, 0, 3, "16 rows x 32 cols x 3 x 32 filters over one window, 256 threads", 1},
    {4, 2, 4, 0, 3, "16 rows x 32 cols x 3 x 64 filters over one window, 256 threads", 1},
    {4, 1, 4, 0, 1, "4 rows x 128 cols x 32 filters, 256 threads, one workgroup per tile", 4},
    {4, 1, 8, 0, 1, "4 rows x 256 cols x 32 filters, 512 threads, one workgroup per tile", 8},
    {4, 1, 4, 0, 3, "4 rows x 128 cols x 3 x 32 filters over one window, 256 threads", 4},
    {4, 1, 8, 0, 1, "8 rows x 128 cols x 32 filters, 512 threads, one workgroup per tile", 4},
    {4, 1, 8, 0, 3, "8 rows x 128 cols x 3 x 32 filters over one window, 512 threads", 4},
};
constexpr int N_TILE_CFGS = (int)(sizeof(TILE_CFGS) / sizeof(TILE_CFGS[0]));
constexpr int MAX_BB = 2;                 // most filter blocks per tile over TILE_CFGS
constexpr int PLACE_CHUNKS = 8;           // dependency chunks of the overlapped strategy
constexpr int MAX_FILTER_H = 16;
constexpr int MAX_FILTER_W = 32;
constexpr int N_MODES = DPMT_CP_FP32 + 1;
constexpr int CP_CHUNKS_PER_TILE = 8;     // 4-filter chunks a CP tile walks over its halo

enum Role { ROLE_ROOT = 0, ROLE_PART = 1, ROLE_ALL = 2 };

struct HostGroup {
    Role role;
    int h, w;
    std::vector<int> filters;   // response-block column order
};

struct ModeData {
    bool ready = false;
    Packing pk{};
    CorrKind kind = CORR_F32;
    void* dG = nullptr;         // packed operands of every group
    GroupDesc* dGroups = nullptr;
    std::vector<GroupDesc> groups;
    float* dU = nullptr;        // 32 x RP projection basis (tensor modes)
    float* dMaster = nullptr;   // FP8: FP32 factors in operand order
    float* dChmax = nullptr;    // FP8: per filter slot, largest |factor| of each channel
    RequantBlock* dRequant = nullptr;
    int n_requant = 0;
    float* dTk = nullptr;       // FP8: per-filter scales
    float* dScales = nullptr;   // FP8: RP channel scales + channel-max scratch
    int max_h = 0, max_S = 0;   // over the groups used by score_pyramid
    int tile_cfg = 0;           // TILE_CFGS entry used by score_pyramid
    // planned correlation tiles per tile shape (rows per tile, filter blocks),
    // valid for plan_id: cost order for batched launches, (image, level) order
    // with ranges for per-level launches
    struct TileSet {
        int plan_id = -1;
        CorrTile* dTiles = nullptr;
        CorrTile* dTilesLvl = nullptr;
        CorrTile* dTilesChunk = nullptr;
        int n_tiles = 0;
        std::vector<std::array<int, 4>> lvl;   // (image, level, begin, end)
        std::vector<std::array<int, 2>> chunk; // (begin, end) into dTilesChunk per chunk
        // per order list (cost, level, chunk): runs of tiles whose groups have
        // the same filter height, (begin, end, height, most K-steps)
        std::array<std::vector<std::array<int, 4>>, 3> runs;
    };
    std::map<std::array<int, 4>, TileSet> tilesets;
    // CP mode: chunk table and packed factors, first chunk of every group,
    // and its tiles (cost order, (image, level) order, chunk order)
    CpChunk* dCpChunks = nullptr;
    float* dCpFac = nullptr;
    std::vector<int> cp_chunk0;
    struct CpTileSet {
        int plan_id = -1;
        CpTile* dTiles = nullptr;
        CpTile* dTilesLvl = nullptr;
        CpTile* dTilesChunk = nullptr;
        int n_tiles = 0;
        size_t lds = 0;
        std::vector<std::array<int, 4>> lvl;
        std::vector<std::array<int, 2>> chunk;
    } cp;
};

void free_tilesets(ModeData& m);

struct LevelInfo {
    int64_t cell_offset;
    int rows, cols;
};

struct BlockKey {
    int img, level, group;
    bool operator<(const BlockKey& o) const {
        return std::tie(img, level, group) < std::tie(o.img, o.level, o.group);
    }
};

struct BlockInfo {
    int64_t off;      // element offset of the group's first plane in the response workspace
    int Ho, Wo;
    int ld;           // plane row pitch (Wo rounded up to a multiple of 4)
    int64_t rng;      // range slot of the group's first plane
};

int pitch_of(int Wo) { return (Wo + 3) & ~3; }

bool is_tensor(dpmt_mode m) { return m >= DPMT_TENSOR_FP32 && m <= DPMT_TENSOR_FP8; }

template <typename T>
hipError_t upload(T** dptr, const std::vector<T>& v) {
    if (*dptr) { (void)hipFree(*dptr); *dptr = nullptr; }
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dptr), v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

// float32 -> bfloat16, round to nearest even (finite inputs)
uint16_t f32_to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

}  // namespace

constexpr int N_STAGES = 3;             // projection, correlation, placement
constexpr int N_EVENTS = N_STAGES + 1;

struct dpmt_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    std::string err;

    // bank
    bool loaded = false;
    std::vector<dpmt_shape> shapes;
    std::vector<int64_t> woff;          // float offset of each filter in `weights`
    std::vector<float> weights;
    struct Comp {
        int root;
        std::vector<int> parts;
        std::vector<std::array<int, 2>> anchors;
        std::vector<std::array<float, 4>> deform;
    };
    std::vector<Comp> comps;
    std::vector<HostGroup> groups;      // root groups, part groups, all groups
    std::vector<int> comp_root_group, comp_root_col;
    std::vector<std::vector<std::pair<int, int>>> comp_part_gc;   // [comp][slot] -> (part group, column)

    // decomposition
    bool decomposed = false;
    int rank = 0;
    std::vector<double> sigma;          // 32
    std::vector<double> Ufull;          // 32 x 32 row major, columns = eigenvectors

    ModeData modes[N_MODES];

    // per-filter CP form: ranks, and factors A (h x R), B (w x R), C (32 x R)
    // row major per filter at cp_off[k]
    bool cp_ready = false;
    std::vector<int> cp_rank;
    std::vector<int64_t> cp_off;
    std::vector<float> cp_fac;
    // convolution shortening: thresholds t_r per filter (R_k each, in filter
    // order) and the rejection bytes the CP correlation writes per response
    bool thr_set = false;
    std::vector<float> cp_thr;
    std::vector<int64_t> thr_off;

    // plan
    int plan_id = 0;
    bool planned = false;
    std::vector<std::vector<LevelInfo>> pyr;
    std::vector<int> octave;
    std::map<BlockKey, BlockInfo> blocks;
    int64_t resp_elems = 0;
    int64_t n_slots = 0;                // response planes (one value range each)
    int64_t n_cells = 0;
    std::vector<int32_t> m_image, m_level, m_comp, m_rows, m_cols;
    std::vector<int64_t> m_score_off, m_offs_off;
    std::vector<MapDesc> maps;
    std::vector<MapPart> map_parts;
    std::vector<int2> place_blk;        // per placement block: (map, strip), work order
    std::vector<int2> place_blk_lvl;    // the same blocks in (image, level) order
    std::vector<std::array<int, 4>> place_lvl;   // (image, level, begin, end) into place_blk_lvl
    // overlapped strategy: (image, root level) dependency groups cut into
    // chunks; a chunk's placement needs only its own correlation tiles
    std::map<std::pair<int, int>, int> chunk_of;  // (image, root level) -> chunk
    int n_chunks = 0;
    std::vector<int2> place_blk_chunk;            // placement blocks in chunk order
    std::vector<std::array<int, 2>> place_chunk;  // (begin, end) per chunk
    // LDS of each launch, sized by its own maps: the batched launch is split
    // into runs of blocks of equal workgroups per CU (place_runs, (begin,
    // end) into place_blk); per-level launches and chunks get their own
    std::vector<std::array<int, 2>> place_runs;
    std::vector<size_t> place_runs_lds, place_lvl_lds, place_chunk_lds;   // dynamic LDS per launch
    dpmt_layout layout{};

    // device workspace
    float* d_resp = nullptr;            // filter response planes
    int* d_rkeys = nullptr;             // 2 * n_slots value-range keys
    void* d_Z = nullptr;
    size_t Z_bytes = 0;
    MapDesc* d_maps = nullptr;
    MapPart* d_parts = nullptr;
    int2* d_place_blk = nullptr;
    int2* d_place_blk_lvl = nullptr;
    int2* d_place_blk_chunk = nullptr;
    int64_t* d_det_counts = nullptr;              // detection compaction scratch
    uint8_t* d_flags = nullptr;                   // rejection bytes, one per response element
    size_t flags_bytes = 0;
    hipStream_t aux_stream = nullptr;             // placement chunks of the overlapped strategy
    std::vector<hipEvent_t> chunk_ev;             // chunk done, fork, join

    // launch strategy and the captured graph of the batched launches
    int launch = DPMT_LAUNCH_BATCHED;
    hipStream_t cap_stream = nullptr;
    struct GraphKey {
        int mode = -1, plan_id = -1, cfg = -1;
        const void* f = nullptr;
        const void* s = nullptr;
        const void* o = nullptr;
        bool operator==(const GraphKey& k) const {
            return mode == k.mode && plan_id == k.plan_id && cfg == k.cfg && f == k.f && s == k.s && o == k.o;
        }
    };
    GraphKey graph_key;
    hipGraphExec_t graph_exec = nullptr;

    // HOG pyramid: level table and work lists of the last geometry, and the
    // histogram scratch (grown as needed)
    std::vector<HogLevelDesc> hog_levels;
    std::vector<int4> hog_tiles;
    std::vector<int2> hog_blocks;
    int hog_H = -1, hog_W = -1;
    HogLevelDesc* d_hog_levels = nullptr;
    int4* d_hog_tiles = nullptr;
    int2* d_hog_blocks = nullptr;
    float* d_hog_hist = nullptr;
    int64_t hog_hist_cells = 0;

    // profiling: one set of events per profiled call
    bool prof = false;
    std::vector<std::array<hipEvent_t, N_EVENTS>> ev_sets;
    std::vector<char> ev_whole_only;    // per set: stages not separable (graph launch)
    int ev_used = 0;

    bool has_device() const { return device >= 0; }
};

namespace {

dpmt_status fail(dpmt_ctx* c, dpmt_status s, const std::string& msg) {
    if (c) c->err = msg;
    else g_free_error = msg;
    return s;
}

dpmt_status hip_fail(dpmt_ctx* c, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? DPMT_E_NOMEM : DPMT_E_DEVICE, m);
}

#define HIP_TRY(ctx, call, what)                          \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

void free_tilesets(ModeData& m) {
    for (auto& kv : m.tilesets) {
        dfree(kv.second.dTiles);
        dfree(kv.second.dTilesLvl);
        dfree(kv.second.dTilesChunk);
    }
    m.tilesets.clear();
    dfree(m.cp.dTiles);
    dfree(m.cp.dTilesLvl);
    dfree(m.cp.dTilesChunk);
    m.cp = ModeData::CpTileSet{};
}

void free_mode(ModeData& m) {
    dfree(m.dMaster);
    dfree(m.dChmax);
    dfree(m.dRequant);
    dfree(m.dTk);
    dfree(m.dScales);
    dfree(m.dG);
    dfree(m.dGroups);
    dfree(m.dU);
    dfree(m.dCpChunks);
    dfree(m.dCpFac);
    free_tilesets(m);
    const int cfg = m.tile_cfg;
    m = ModeData{};
    m.tile_cfg = cfg;
}

void drop_graph(dpmt_ctx* c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    c->graph_key = dpmt_ctx::GraphKey{};
}

void free_plan(dpmt_ctx* c) {
    dfree(c->d_resp); c->d_resp = nullptr;
    dfree(c->d_rkeys); c->d_rkeys = nullptr;
    dfree(c->d_Z); c->d_Z = nullptr; c->Z_bytes = 0;
    dfree(c->d_maps); c->d_maps = nullptr;
    dfree(c->d_parts); c->d_parts = nullptr;
    dfree(c->d_place_blk); c->d_place_blk = nullptr;
    dfree(c->d_place_blk_lvl); c->d_place_blk_lvl = nullptr;
    dfree(c->d_place_blk_chunk); c->d_place_blk_chunk = nullptr;
    dfree(c->d_det_counts); c->d_det_counts = nullptr;
    dfree(c->d_flags); c->d_flags = nullptr; c->flags_bytes = 0;
    for (auto& m : c->modes) free_tilesets(m);
    drop_graph(c);
    c->planned = false;
}

// Channels padded to what the operand packing supports.
int padded_rank(dpmt_mode mode, int R) {
    if (mode == DPMT_DIRECT_FP32) return 32;
    if (mode == DPMT_TENSOR_FP8) return R <= 16 ? 16 : 32;
    if (R <= 4) return 4;
    if (R <= 8) return 8;
    if (R <= 16) return 16;
    if (mode == DPMT_TENSOR_FP32 && R <= 24) return 24;
    return 32;
}

Packing packing_for(dpmt_mode mode, int R) {
    Packing p{};
    p.RP = padded_rank(mode, R);
    p.esz = (mode == DPMT_TENSOR_BF16) ? 2 : (mode == DPMT_TENSOR_FP8 ? 1 : 4);
    p.PB = std::min(p.RP * p.esz, 32);
    p.Q = p.RP * p.esz / p.PB;
    return p;
}

// Jacobi eigen-decomposition of a symmetric 32x32 matrix (cyclic sweeps of
// plane rotations; Golub & Van Loan, Section 8.5).  A is destroyed; on return
// its diagonal holds the eigenvalues and V (row major) the eigenvectors as
// columns.
void jacobi_eigen(std::vector<double>& A, std::vector<double>& V, int n) {
    V.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    double fro = 0;
    for (double x : A) fro += x * x;
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += 2 * A[p * n + q] * A[p * n + q];
        if (std::sqrt(off) <= 1e-15 * fro || fro == 0) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double app = A[p * n + p], aqq = A[q * n + q];
                const double theta = (aqq - app) / (2 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
                const double cs = 1.0 / std::sqrt(t * t + 1), sn = t * cs;
                for (int k = 0; k < n; ++k) {        // A <- A J  (columns p, q)
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = cs * akp - sn * akq;
                    A[k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {        // A <- J^T A  (rows p, q)
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = cs * apk - sn * aqk;
                    A[q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {        // V <- V J
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = cs * vkp - sn * vkq;
                    V[k * n + q] = sn * vkp + cs * vkq;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Per-filter CP form by alternating least squares (Section 4), FP64.
// The tensor is n1 x n2 x n3 row major (f[i][j][k] at (i * n2 + j) * n3 + k);
// factors are row major n_d x R.
// ---------------------------------------------------------------------------
struct CpFit {
    std::vector<double> A, B, C;
    double rel_err = 0;
};

// Symmetric pseudo-inverse of an R x R positive semi-definite matrix:
// eigenvalues below 1e-13 of the largest are treated as zero.
std::vector<double> psd_pinv(std::vector<double> G, int R) {
    std::vector<double> V;
    jacobi_eigen(G, V, R);
    double lmax = 0;
    for (int i = 0; i < R; ++i) lmax = std::max(lmax, G[i * R + i]);
    std::vector<double> P((size_t)R * R, 0.0);
    for (int e = 0; e < R; ++e) {
        const double l = G[e * R + e];
        if (!(l > 1e-13 * lmax)) continue;
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < R; ++j) P[i * R + j] += V[i * R + e] * V[j * R + e] / l;
    }
    return P;
}

// Starting factor for mode d: leading R left singular vectors of the mode-d
// unfolding (eigenvectors of its Gram matrix by decreasing eigenvalue); the
// columns beyond the mode size are filled with a fixed pseudo-random pattern
// (zero columns would stay zero under the updates).
std::vector<double> cp_start(const std::vector<double>& G, int n, int R) {
    std::vector<double> g = G, V;
    jacobi_eigen(g, V, n);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return g[a * n + a] > g[b * n + b]; });
    std::vector<double> F((size_t)n * R, 0.0);
    for (int r = 0; r < R; ++r)
        for (int i = 0; i < n; ++i) {
            if (r < n) {
                F[(size_t)i * R + r] = V[i * n + order[r]];
            } else {
                uint64_t z = (uint64_t)(r * 131 + i) * 0x9E3779B97F4A7C15ull;
                z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;
                z ^= z >> 29;
                F[(size_t)i * R + r] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
            }
        }
    return F;
}

// One mode update: F = M (Gram_1 * Gram_2)^+, M the MTTKRP of that mode.
void cp_solve(std::vector<double>& F, const std::vector<double>& M, const std::vector<double>& P1,
              const std::vector<double>& P2, int n, int R) {
    std::vector<double> G((size_t)R * R);
    for (int i = 0; i < R * R; ++i) G[i] = P1[i] * P2[i];
    const std::vector<double> Gi = psd_pinv(G, R);
    for (int i = 0; i < n; ++i)
        for (int r = 0; r < R; ++r) {
            double v = 0;
            for (int q = 0; q < R; ++q) v += M[(size_t)i * R + q] * Gi[q * R + r];
            F[(size_t)i * R + r] = v;
        }
}

std::vector<double> gram_cols(const std::vector<double>& F, int n, int R) {
    std::vector<double> G((size_t)R * R, 0.0);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < R; ++a)
            for (int b = 0; b < R; ++b) G[a * R + b] += F[(size_t)i * R + a] * F[(size_t)i * R + b];
    return G;
}

CpFit cp_als(const float* f32, int n1, int n2, int n3, int R, int max_iters, double tol) {
    const size_t N = (size_t)n1 * n2 * n3;
    std::vector<double> f(f32, f32 + N);
    double nf2 = 0;
    for (double v : f) nf2 += v * v;
    const double nf = std::sqrt(nf2);
    // Gram matrices of the three unfoldings for the starting factors
    std::vector<double> G1((size_t)n1 * n1, 0.0), G2((size_t)n2 * n2, 0.0), G3((size_t)n3 * n3, 0.0);
    auto at = [&](int i, int j, int k) { return f[((size_t)i * n2 + j) * n3 + k]; };
    for (int i = 0; i < n1; ++i)
        for (int i2 = 0; i2 < n1; ++i2) {
            double v = 0;
            for (int j = 0; j < n2; ++j)
                for (int k = 0; k < n3; ++k) v += at(i, j, k) * at(i2, j, k);
            G1[i * n1 + i2] = v;
        }
    for (int j = 0; j < n2; ++j)
        for (int j2 = 0; j2 < n2; ++j2) {
            double v = 0;
            for (int i = 0; i < n1; ++i)
                for (int k = 0; k < n3; ++k) v += at(i, j, k) * at(i, j2, k);
            G2[j * n2 + j2] = v;
        }
    for (int k = 0; k < n3; ++k)
        for (int k2 = 0; k2 < n3; ++k2) {
            double v = 0;
            for (int i = 0; i < n1; ++i)
                for (int j = 0; j < n2; ++j) v += at(i, j, k) * at(i, j, k2);
            G3[k * n3 + k2] = v;
        }
    CpFit fit;
    fit.A = cp_start(G1, n1, R);
    fit.B = cp_start(G2, n2, R);
    fit.C = cp_start(G3, n3, R);
    std::vector<double>& A = fit.A;
    std::vector<double>& B = fit.B;
    std::vector<double>& C = fit.C;
    std::vector<double> M;
    auto error = [&]() {
        double e2 = 0;
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j)
                for (int k = 0; k < n3; ++k) {
                    double v = 0;
                    for (int r = 0; r < R; ++r) v += A[(size_t)i * R + r] * B[(size_t)j * R + r] * C[(size_t)k * R + r];
                    const double d = at(i, j, k) - v;
                    e2 += d * d;
                }
        return std::sqrt(e2);
    };
    double prev = -1;
    for (int it = 0; it < max_iters; ++it) {
        // A: M[i][r] = sum_jk f[i][j][k] B[j][r] C[k][r]
        M.assign((size_t)n1 * R, 0.0);
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j)
                for (int k = 0; k < n3; ++k) {
                    const double v = at(i, j, k);
                    for (int r = 0; r < R; ++r) M[(size_t)i * R + r] += v * B[(size_t)j * R + r] * C[(size_t)k * R + r];
                }
        cp_solve(A, M, gram_cols(B, n2, R), gram_cols(C, n3, R), n1, R);
        M.assign((size_t)n2 * R, 0.0);
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j)
                for (int k = 0; k < n3; ++k) {
                    const double v = at(i, j, k);
                    for (int r = 0; r < R; ++r) M[(size_t)j * R + r] += v * A[(size_t)i * R + r] * C[(size_t)k * R + r];
                }
        cp_solve(B, M, gram_cols(A, n1, R), gram_cols(C, n3, R), n2, R);
        M.assign((size_t)n3 * R, 0.0);
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j)
                for (int k = 0; k < n3; ++k) {
                    const double v = at(i, j, k);
                    for (int r = 0; r < R; ++r) M[(size_t)k * R + r] += v * A[(size_t)i * R + r] * B[(size_t)j * R + r];
                }
        cp_solve(C, M, gram_cols(A, n1, R), gram_cols(B, n2, R), n3, R);
        const double err = error();
        if (err <= tol * nf) break;
        if (prev >= 0 && prev - err <= 1e-12 * prev) break;
        prev = err;
    }
    // balance the three factor norms of every term (the tensor is unchanged)
    for (int r = 0; r < R; ++r) {
        double na = 0, nb = 0, nc = 0;
        for (int i = 0; i < n1; ++i) na += A[(size_t)i * R + r] * A[(size_t)i * R + r];
        for (int j = 0; j < n2; ++j) nb += B[(size_t)j * R + r] * B[(size_t)j * R + r];
        for (int k = 0; k < n3; ++k) nc += C[(size_t)k * R + r] * C[(size_t)k * R + r];
        na = std::sqrt(na);
        nb = std::sqrt(nb);
        nc = std::sqrt(nc);
        if (na == 0 || nb == 0 || nc == 0) continue;
        const double g = std::cbrt(na * nb * nc);
        for (int i = 0; i < n1; ++i) A[(size_t)i * R + r] *= g / na;
        for (int j = 0; j < n2; ++j) B[(size_t)j * R + r] *= g / nb;
        for (int k = 0; k < n3; ++k) C[(size_t)k * R + r] *= g / nc;
    }
    fit.rel_err = nf > 0 ? error() / nf : 0.0;
    return fit;
}

// Operand weights of filter k for a mode: h x w x RP values in float64
// (original weights for the direct mode, G_k = f_k x_3 U_R for tensor modes).
std::vector<double> operand_weights(const dpmt_ctx* c, int k, const Packing& pk, bool tensor) {
    const int h = c->shapes[k].h, w = c->shapes[k].w;
    const float* f = c->weights.data() + c->woff[k];
    std::vector<double> out((size_t)h * w * pk.RP, 0.0);
    for (int cell = 0; cell < h * w; ++cell) {
        if (!tensor) {
            for (int l = 0; l < 32; ++l) out[(size_t)cell * pk.RP + l] = f[cell * 32 + l];
        } else {
            for (int r = 0; r < c->rank; ++r) {
                double s = 0;
                for (int l = 0; l < 32; ++l) s += (double)f[cell * 32 + l] * c->Ufull[l * 32 + r];
                out[(size_t)cell * pk.RP + r] = s;
            }
        }
    }
    return out;
}

// Pack every group's operand in MFMA B-fragment order:
// [block][plane q][step s][filter row n][lane 0..63][FB bytes], lane = f + 32*j
// holding bytes [2FB s + FB j, 2FB s + FB j + FB) of filter (32*block + f)'s
// flattened plane-q row n (w cells x PB bytes, zero beyond).  FB is the
// fragment width: 16 bytes for FP32/BF16, 32 for FP8.  FP8 operands are made
// on the device at every call (their scales depend on the features), from an
// FP32 master copy in the same element order.
// CP mode: every group cut into chunks of 4 filter columns; per chunk the
// channel factors in MFMA B-operand order (batches of 4 filters x 4 terms),
// then each filter's row and column factors transposed (a_r[n] at r*h + n,
// then b_r[m] at R*h + r*w + m).
dpmt_status prepare_cp(dpmt_ctx* c) {
    ModeData& md = c->modes[DPMT_CP_FP32];
    if (md.ready) return DPMT_OK;
    if (!c->cp_ready) return fail(c, DPMT_E_STATE, "CP mode needs dpmt_decompose_cp or dpmt_load_cp first");
    std::vector<CpChunk> chunks;
    std::vector<float> fac;
    md.cp_chunk0.assign(c->groups.size(), 0);
    md.max_h = 0;
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        const HostGroup& hg = c->groups[gi];
        md.cp_chunk0[gi] = (int)chunks.size();
        if (hg.role != ROLE_ALL) md.max_h = std::max(md.max_h, hg.h);
        const int ng = (int)hg.filters.size();
        for (int f0 = 0; f0 < ng; f0 += 4) {
            CpChunk ch{};
            int kk[4] = {-1, -1, -1, -1};
            for (int j = 0; j < 4; ++j)
                if (f0 + j < ng) {
                    kk[j] = hg.filters[f0 + j];
                    ch.R[j] = c->cp_rank[kk[j]];
                    ch.nq = std::max(ch.nq, (ch.R[j] + 3) / 4);
                }
            ch.c_off = (int64_t)fac.size();
            fac.resize(fac.size() + (size_t)ch.nq * 64 * 8, 0.f);
            for (int q = 0; q < ch.nq; ++q)
                for (int lane = 0; lane < 64; ++lane) {
                    const int col = lane & 15, j = col >> 2, r = 4 * q + (col & 3);
                    if (kk[j] < 0 || r >= ch.R[j]) continue;
                    const int k = kk[j], R = ch.R[j];
                    const float* Ck = c->cp_fac.data() + c->cp_off[k] + (int64_t)(hg.h + hg.w) * R;
                    for (int st = 0; st < 8; ++st)
                        fac[ch.c_off + ((size_t)q * 64 + lane) * 8 + st] = Ck[(8 * (lane >> 4) + st) * R + r];
                }
            for (int j = 0; j < 4; ++j) {
                if (kk[j] < 0) continue;
                const int k = kk[j], R = ch.R[j];
                const float* Ak = c->cp_fac.data() + c->cp_off[k];
                const float* Bk = Ak + (int64_t)hg.h * R;
                ch.ab_off[j] = (int64_t)fac.size();
                for (int r = 0; r < R; ++r)
                    for (int n = 0; n < hg.h; ++n) fac.push_back(Ak[n * R + r]);
                for (int r = 0; r < R; ++r)
                    for (int m = 0; m < hg.w; ++m) fac.push_back(Bk[m * R + r]);
                if (c->thr_set)
                    for (int r = 0; r < R; ++r) fac.push_back(c->cp_thr[c->thr_off[k] + r]);
            }
            chunks.push_back(ch);
        }
    }
    fac.resize(fac.size() + 8, 0.f);
    if (c->has_device()) {
        HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
        HIP_TRY(c, upload(&md.dCpChunks, chunks), "upload CP chunk table");
        HIP_TRY(c, upload(&md.dCpFac, fac), "upload CP factors");
    }
    md.ready = true;
    return DPMT_OK;
}

dpmt_status prepare_mode(dpmt_ctx* c, dpmt_mode mode) {
    if (mode == DPMT_CP_FP32) return prepare_cp(c);
    ModeData& md = c->modes[mode];
    if (md.ready) return DPMT_OK;
    const bool tensor = mode != DPMT_DIRECT_FP32;
    const bool fp8 = mode == DPMT_TENSOR_FP8;
    if (tensor && !c->decomposed) return fail(c, DPMT_E_STATE, "tensor mode needs dpmt_decompose first");
    md.pk = packing_for(mode, c->rank);
    md.kind = (mode == DPMT_TENSOR_BF16) ? CORR_BF16 : (fp8 ? CORR_FP8 : CORR_F32);
    const Packing pk = md.pk;
    const int FB = fp8 ? 32 : 16;
    const int KS = 2 * FB;
    std::vector<unsigned char> G;       // FP32 / BF16 operand bytes
    std::vector<float> master;          // FP8: FP32 values in operand element order
    std::vector<RequantBlock> rq;
    int t_slots = 0;
    md.groups.clear();
    md.max_h = md.max_S = 0;
    std::vector<std::vector<double>> opw(c->shapes.size());
    for (size_t gi = 0; gi < c->groups.size(); ++gi) {
        const HostGroup& hg = c->groups[gi];
        GroupDesc gd{};
        gd.h = hg.h;
        gd.w = hg.w;
        gd.ng = (int)hg.filters.size();
        gd.S = (hg.w * pk.PB + KS - 1) / KS;
        const int nblk = (gd.ng + 31) / 32;
        const int nblk_pad = (nblk + MAX_BB - 1) / MAX_BB * MAX_BB;   // a tile may read MAX_BB blocks
        const size_t chunk = (size_t)64 * FB;      // bytes per (block, plane, step, row)
        const size_t blk_bytes = (size_t)pk.Q * gd.S * gd.h * chunk;
        const size_t base_elems = fp8 ? master.size() : G.size();
        gd.g_off = (int64_t)base_elems;               // byte offset (FP8: one byte per element)
        gd.t_off = t_slots;
        t_slots += nblk_pad * 32;
        if (hg.role != ROLE_ALL) {
            md.max_h = std::max(md.max_h, gd.h);
            md.max_S = std::max(md.max_S, gd.S);
        }
        if (fp8) master.resize(master.size() + nblk_pad * blk_bytes, 0.f);
        else G.resize(G.size() + nblk_pad * blk_bytes, 0);
        for (int b = 0; b < nblk_pad && fp8; ++b) {
            RequantBlock r{};
            r.m_off = (int64_t)(base_elems + b * blk_bytes);
            r.g_off = (int64_t)(base_elems + b * blk_bytes);
            r.chunks = pk.Q * gd.S * gd.h;
            r.h = gd.h;
            r.S = gd.S;
            r.ng = gd.ng;
            r.f0 = b * 32;
            r.t_off = gd.t_off + b * 32;
            rq.push_back(r);
        }
        for (int fi = 0; fi < gd.ng; ++fi) {
            const int k = hg.filters[fi];
            if (opw[k].empty()) opw[k] = operand_weights(c, k, pk, tensor);
            const std::vector<double>& wv = opw[k];
            const int blk = fi / 32, f = fi % 32;
            for (int q = 0; q < pk.Q; ++q)
                for (int sx = 0; sx < gd.S; ++sx)
                    for (int n = 0; n < gd.h; ++n)
                        for (int j = 0; j < 2; ++j) {
                            const size_t unit = base_elems + blk * blk_bytes +
                                                (((size_t)q * gd.S + sx) * gd.h + n) * chunk +
                                                (size_t)(f + 32 * j) * FB;
                            for (int e = 0; e < FB / pk.esz; ++e) {
                                const int o = KS * sx + FB * j + e * pk.esz;   // flattened byte
                                const int m = o / pk.PB;
                                const int ch = q * (pk.PB / pk.esz) + (o % pk.PB) / pk.esz;
                                if (m >= gd.w) continue;
                                const double v = wv[((size_t)n * gd.w + m) * pk.RP + ch];
                                if (fp8) {
                                    master[unit + e] = (float)v;
                                } else if (pk.esz == 4) {
                                    const float fv = (float)v;
                                    std::memcpy(G.data() + unit + e * 4, &fv, 4);
                                } else {
                                    const uint16_t bv = f32_to_bf16((float)v);
                                    std::memcpy(G.data() + unit + e * 2, &bv, 2);
                                }
                            }
                        }
        }
        md.groups.push_back(gd);
    }
    // FP8: the largest |factor| of every channel of every filter slot, in the
    // operand order the requantisation walks (element e of unit u of a block
    // is channel q * PB + (64 sidx + 32 (lane / 32) + e) % PB)
    std::vector<float> chmax;
    if (fp8) {
        chmax.assign((size_t)std::max(t_slots, 1) * pk.RP, 0.f);
        for (const RequantBlock& r : rq)
            for (int u = 0; u < r.chunks * 64; ++u) {
                const int lane = u & 63, ch = u >> 6;
                const int sidx = (ch / r.h) % r.S, q = (ch / r.h) / r.S;
                float* mk = chmax.data() + (size_t)(r.t_off + (lane & 31)) * pk.RP;
                for (int e = 0; e < 32; ++e) {
                    const int o = (64 * sidx + 32 * (lane >> 5) + e) % pk.PB;
                    float& m = mk[q * pk.PB + o];
                    m = std::max(m, std::fabs(master[(size_t)r.m_off + (size_t)u * 32 + e]));
                }
            }
    }
    if (c->has_device()) {
        HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
        HIP_TRY(c, upload(&md.dGroups, md.groups), "upload group table");
        if (fp8) {
            HIP_TRY(c, upload(&md.dMaster, master), "upload FP8 master factors");
            HIP_TRY(c, upload(&md.dChmax, chmax), "upload FP8 channel maxima");
            HIP_TRY(c, upload(&md.dRequant, rq), "upload requant table");
            md.n_requant = (int)rq.size();
            HIP_TRY(c, hipMalloc(&md.dG, std::max<size_t>(master.size(), 16)), "allocate FP8 operand");
            HIP_TRY(c, hipMalloc((void**)&md.dTk, (size_t)std::max(t_slots, 1) * 4), "allocate FP8 filter scales");
            HIP_TRY(c, hipMalloc((void**)&md.dScales, (size_t)(pk.RP + FP8_PARTIALS) * 4), "allocate FP8 channel scales");
        } else {
            HIP_TRY(c, upload(reinterpret_cast<unsigned char**>(&md.dG), G), "upload packed filters");
        }
        if (tensor) {
            std::vector<float> U((size_t)32 * pk.RP, 0.f);
            for (int l = 0; l < 32; ++l)
                for (int r = 0; r < c->rank; ++r) U[l * pk.RP + r] = (float)c->Ufull[l * 32 + r];
            HIP_TRY(c, upload(&md.dU, U), "upload basis");
        }
    }
    md.ready = true;
    return DPMT_OK;
}

// FP8 mode: channel maxima of the given cells, channel scales and the
// requantised factors; then the scaled projection of cells into Z.
// rkeys (may be NULL): value-range keys reset along the way.
hipError_t fp8_prepare(ModeData& md, const float* X, int64_t n_cells, int* rkeys, int64_t n_slots,
                       hipStream_t st) {
    return launch_fp8_prepare(X, n_cells, md.dU, md.pk.RP, md.dScales + md.pk.RP, md.dScales,
                              md.dRequant, md.n_requant, md.dMaster, md.dChmax, static_cast<uint8_t*>(md.dG),
                              md.dTk, rkeys, n_slots, st);
}

hipError_t fp8_operands(ModeData& md, const float* X, int64_t n_cells, void* Z, int* rkeys, int64_t n_slots,
                        hipStream_t st) {
    hipError_t e = fp8_prepare(md, X, n_cells, rkeys, n_slots, st);
    if (e != hipSuccess) return e;
    return launch_project_fp8(X, n_cells, md.dU, md.pk.RP, md.dScales, Z, st);
}

void build_groups(dpmt_ctx* c) {
    c->groups.clear();
    c->comp_root_group.assign(c->comps.size(), -1);
    c->comp_root_col.assign(c->comps.size(), -1);
    std::map<std::pair<int, int>, int> root_g, part_g, all_g;
    auto group_for = [&](std::map<std::pair<int, int>, int>& gm, Role role, int k) {
        const auto key = std::make_pair(c->shapes[k].h, c->shapes[k].w);
        auto it = gm.find(key);
        if (it != gm.end()) return it->second;
        c->groups.push_back(HostGroup{role, key.first, key.second, {}});
        gm[key] = (int)c->groups.size() - 1;
        return (int)c->groups.size() - 1;
    };
    auto col_of = [&](int g, int k) {
        auto& fl = c->groups[g].filters;
        auto it = std::find(fl.begin(), fl.end(), k);
        if (it != fl.end()) return (int)(it - fl.begin());
        fl.push_back(k);
        return (int)fl.size() - 1;
    };
    for (size_t ci = 0; ci < c->comps.size(); ++ci) {
        const int g = group_for(root_g, ROLE_ROOT, c->comps[ci].root);
        c->comp_root_group[ci] = g;
        c->comp_root_col[ci] = col_of(g, c->comps[ci].root);
    }
    c->comp_part_gc.assign(c->comps.size(), {});
    for (size_t ci = 0; ci < c->comps.size(); ++ci)
        for (int k : c->comps[ci].parts) {
            const int g = group_for(part_g, ROLE_PART, k);
            c->comp_part_gc[ci].push_back({g, col_of(g, k)});
        }
    for (size_t k = 0; k < c->shapes.size(); ++k) {
        const int g = group_for(all_g, ROLE_ALL, (int)k);
        col_of(g, (int)k);
    }
}

void add_tiles(std::vector<CorrTile>& tiles, const GroupDesc& gd, int group, int64_t z_cell,
               int64_t out_off, int rng, int H, int W, int rows, int cols, int bb, int nfb) {
    const int Ho = H - gd.h + 1, Wo = W - gd.w + 1;
    if (Ho <= 0 || Wo <= 0) return;
    const int nblk = (gd.ng + 31) / 32;
    for (int y0 = 0; y0 < Ho; y0 += rows)
        for (int x0 = 0; x0 < Wo; x0 += cols)
            for (int fb = 0; fb < nblk; fb += bb * nfb) {
                CorrTile t{};
                t.z_cell = z_cell;
                t.out_off = out_off;
                t.H = H;
                t.W = W;
                t.Ho = Ho;
                t.Wo = Wo;
                t.ld = pitch_of(Wo);
                t.rng = rng;
                t.y0 = y0;
                t.x0 = x0;
                t.fb0 = fb;
                t.group = group;
                t.nfb = std::min(nfb, (nblk - fb + bb - 1) / bb);
                tiles.push_back(t);
            }
}

// Correlation tiles of the mode's tile configuration for the current plan.
dpmt_status prepare_tiles(dpmt_ctx* c, dpmt_mode mode, ModeData::TileSet** out) {
    ModeData& md = c->modes[mode];
    const TileCfg& tc = TILE_CFGS[md.tile_cfg];
    const std::array<int, 4> key{tc.ty * (tc.wy / tc.wx), tc.bb, tc.nfb, 32 * tc.wx};
    ModeData::TileSet& ts = md.tilesets[key];
    *out = &ts;
    if (ts.plan_id == c->plan_id && (ts.dTiles || ts.n_tiles == 0)) return DPMT_OK;
    dfree(ts.dTiles);
    dfree(ts.dTilesLvl);
    ts = ModeData::TileSet{};
    std::vector<CorrTile> tiles;                   // blocks are ordered by (image, level, group)
    for (const auto& kv : c->blocks) {
        const BlockKey& k = kv.first;
        const LevelInfo& lv = c->pyr[k.img][k.level];
        const size_t b0 = tiles.size();
        add_tiles(tiles, md.groups[k.group], k.group, lv.cell_offset, kv.second.off,
                  (int)kv.second.rng, lv.rows, lv.cols, key[0], key[3], key[1], key[2]);
        if (tiles.size() == b0) continue;
        if (!ts.lvl.empty() && ts.lvl.back()[0] == k.img && ts.lvl.back()[1] == k.level)
            ts.lvl.back()[3] = (int)tiles.size();
        else
            ts.lvl.push_back({k.img, k.level, (int)b0, (int)tiles.size()});
    }
    if (tiles.size() > (size_t)INT32_MAX) return fail(c, DPMT_E_UNSUPPORTED, "batch too large for one launch");
    // runs of consecutive tiles with equal filter height in one order list
    auto height_runs = [&](const std::vector<CorrTile>& tl) {
        std::vector<std::array<int, 4>> r;
        for (size_t i = 0; i < tl.size(); ++i) {
            const GroupDesc& gd = md.groups[tl[i].group];
            if (!r.empty() && r.back()[2] == gd.h && r.back()[1] == (int)i) {
                r.back()[1] = (int)i + 1;
                r.back()[3] = std::max(r.back()[3], gd.S);
            } else {
                r.push_back({(int)i, (int)i + 1, gd.h, gd.S});
            }
        }
        return r;
    };
    ts.runs[1] = height_runs(tiles);
    HIP_TRY(c, upload(&ts.dTilesLvl, tiles), "upload tiles");
    {   // chunk order for the overlapped strategy, most expensive first within a chunk
        std::vector<std::pair<int, CorrTile>> keyed;
        keyed.reserve(tiles.size());
        for (const auto& r : ts.lvl)                       // tiles of (image r[0], level r[1])
            for (int i = r[2]; i < r[3]; ++i) {
                const CorrTile& t = tiles[i];
                const bool root = c->groups[t.group].role == ROLE_ROOT;
                auto it = c->chunk_of.find({r[0], root ? r[1] : r[1] + c->octave[r[0]]});
                keyed.push_back({it == c->chunk_of.end() ? 0 : it->second, t});
            }
        std::stable_sort(keyed.begin(), keyed.end(), [&](const std::pair<int, CorrTile>& a,
                                                         const std::pair<int, CorrTile>& b) {
            if (a.first != b.first) return a.first < b.first;
            const GroupDesc& ga = md.groups[a.second.group];
            const GroupDesc& gb = md.groups[b.second.group];
            if (ga.h != gb.h) return ga.h > gb.h;
            return (int64_t)ga.h * ga.S > (int64_t)gb.h * gb.S;
        });
        std::vector<CorrTile> ct;
        ct.reserve(keyed.size());
        // within a chunk, taller filters first, then the longer K loops
        ts.chunk.assign(std::max(c->n_chunks, 1), {0, 0});
        for (size_t i = 0; i < keyed.size(); ++i) {
            if (i == 0 || keyed[i].first != keyed[i - 1].first) ts.chunk[keyed[i].first][0] = (int)i;
            ts.chunk[keyed[i].first][1] = (int)i + 1;
            ct.push_back(keyed[i].second);
        }
        ts.runs[2] = height_runs(ct);
        HIP_TRY(c, upload(&ts.dTilesChunk, ct), "upload tiles");
    }
    // taller filters first, then the most expensive groups, so that the tail of
    // the batched launch is short tiles and every filter height is one run
    std::stable_sort(tiles.begin(), tiles.end(), [&](const CorrTile& a, const CorrTile& b) {
        const GroupDesc& ga = md.groups[a.group];
        const GroupDesc& gb = md.groups[b.group];
        if (ga.h != gb.h) return ga.h > gb.h;
        return (int64_t)ga.h * ga.S > (int64_t)gb.h * gb.S;
    });
    ts.runs[0] = height_runs(tiles);
    HIP_TRY(c, upload(&ts.dTiles, tiles), "upload tiles");
    ts.n_tiles = (int)tiles.size();
    ts.plan_id = c->plan_id;
    return DPMT_OK;
}

// CP tiles of one (level, group) block: 32 output columns by as many rows as
// the 1024-cell halo allows, each walking up to CP_CHUNKS_PER_TILE chunks.
void add_cp_tiles(std::vector<CpTile>& tiles, const HostGroup& hg, int chunk0, int64_t x_cell,
                  int64_t out_off, int rng, int H, int W) {
    const int Ho = H - hg.h + 1, Wo = W - hg.w + 1;
    if (Ho <= 0 || Wo <= 0) return;
    const int HX = cp_halo_cols(hg.w), HY = cp_halo_rows(hg.w), TYo = HY - hg.h + 1;
    const int nch = ((int)hg.filters.size() + 3) / 4;
    for (int y0 = 0; y0 < Ho; y0 += TYo)
        for (int x0 = 0; x0 < Wo; x0 += CP_TX)
            for (int q = 0; q < nch; q += CP_CHUNKS_PER_TILE) {
                CpTile t{};
                t.x_cell = x_cell;
                t.out_off = out_off;
                t.H = H;
                t.W = W;
                t.Ho = Ho;
                t.Wo = Wo;
                t.ld = pitch_of(Wo);
                t.rng = rng;
                t.y0 = y0;
                t.x0 = x0;
                t.h = hg.h;
                t.w = hg.w;
                t.HY = HY;
                t.HX = HX;
                t.chunk0 = chunk0 + q;
                t.nchunk = std::min(CP_CHUNKS_PER_TILE, nch - q);
                t.col0 = 4 * q;
                tiles.push_back(t);
            }
}

// CP tiles for the current plan, in the three orders of the launch strategies.
dpmt_status prepare_cp_tiles(dpmt_ctx* c, ModeData::CpTileSet** out) {
    ModeData& md = c->modes[DPMT_CP_FP32];
    ModeData::CpTileSet& ts = md.cp;
    *out = &ts;
    if (ts.plan_id == c->plan_id && (ts.dTiles || ts.n_tiles == 0)) return DPMT_OK;
    dfree(ts.dTiles);
    dfree(ts.dTilesLvl);
    dfree(ts.dTilesChunk);
    ts = ModeData::CpTileSet{};
    std::vector<CpTile> tiles;                     // blocks are ordered by (image, level, group)
    std::vector<int> chunk_key;                    // per tile: dependency chunk of the overlapped strategy
    for (const auto& kv : c->blocks) {
        const BlockKey& k = kv.first;
        const LevelInfo& lv = c->pyr[k.img][k.level];
        const HostGroup& hg = c->groups[k.group];
        const size_t b0 = tiles.size();
        add_cp_tiles(tiles, hg, md.cp_chunk0[k.group], lv.cell_offset, kv.second.off, (int)kv.second.rng,
                     lv.rows, lv.cols);
        if (tiles.size() == b0) continue;
        auto it = c->chunk_of.find({k.img, hg.role == ROLE_ROOT ? k.level : k.level + c->octave[k.img]});
        chunk_key.resize(tiles.size(), it == c->chunk_of.end() ? 0 : it->second);
        if (!ts.lvl.empty() && ts.lvl.back()[0] == k.img && ts.lvl.back()[1] == k.level)
            ts.lvl.back()[3] = (int)tiles.size();
        else
            ts.lvl.push_back({k.img, k.level, (int)b0, (int)tiles.size()});
    }
    if (tiles.size() > (size_t)INT32_MAX) return fail(c, DPMT_E_UNSUPPORTED, "batch too large for one launch");
    for (const CpTile& t : tiles) ts.lds = std::max(ts.lds, cp_lds_bytes(t.HX, t.HY));
    HIP_TRY(c, upload(&ts.dTilesLvl, tiles), "upload CP tiles");
    auto cost = [](const CpTile& t) { return (int64_t)t.h * t.w; };
    {   // chunk order for the overlapped strategy, most expensive first within a chunk
        std::vector<int> idx(tiles.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            if (chunk_key[a] != chunk_key[b]) return chunk_key[a] < chunk_key[b];
            return cost(tiles[a]) > cost(tiles[b]);
        });
        std::vector<CpTile> ct;
        ct.reserve(idx.size());
        ts.chunk.assign(std::max(c->n_chunks, 1), {0, 0});
        for (size_t j = 0; j < idx.size(); ++j) {
            const int ck = chunk_key[idx[j]];
            if (j == 0 || ck != chunk_key[idx[j - 1]]) ts.chunk[ck][0] = (int)j;
            ts.chunk[ck][1] = (int)j + 1;
            ct.push_back(tiles[idx[j]]);
        }
        HIP_TRY(c, upload(&ts.dTilesChunk, ct), "upload CP tiles");
    }
    std::stable_sort(tiles.begin(), tiles.end(), [&](const CpTile& a, const CpTile& b) { return cost(a) > cost(b); });
    HIP_TRY(c, upload(&ts.dTiles, tiles), "upload CP tiles");
    ts.n_tiles = (int)tiles.size();
    ts.plan_id = c->plan_id;
    return DPMT_OK;
}

dpmt_status score_checks(dpmt_ctx* c, dpmt_mode mode, const float* features_dev,
                         const float* scores_dev) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (mode < DPMT_DIRECT_FP32 || mode > DPMT_CP_FP32) return fail(c, DPMT_E_INVALID, "unknown mode");
    if (!c->loaded) return fail(c, DPMT_E_STATE, "score call before dpmt_load_filters");
    if (is_tensor(mode) && !c->decomposed) return fail(c, DPMT_E_STATE, "tensor mode needs dpmt_decompose first");
    if (mode == DPMT_CP_FP32 && !c->cp_ready) return fail(c, DPMT_E_STATE, "CP mode needs dpmt_decompose_cp or dpmt_load_cp first");
    if (!c->planned) return fail(c, DPMT_E_STATE, "score call before dpmt_plan");
    if (!c->has_device()) return fail(c, DPMT_E_STATE, "host-only context cannot score");
    if (!features_dev || (!scores_dev && c->layout.n_score > 0)) return fail(c, DPMT_E_INVALID, "features_dev and scores_dev are required");
    return DPMT_OK;
}

// Algorithm 1's early exit applies to the CP form once thresholds are set.
bool pruning(const dpmt_ctx* c, dpmt_mode mode) { return mode == DPMT_CP_FP32 && c->thr_set; }

// Operands, tiles and the projected-feature buffer of a mode for the plan;
// allocates, so it never runs while a graph is being captured.
dpmt_status score_prepare(dpmt_ctx* c, dpmt_mode mode, hipStream_t st) {
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    dpmt_status s = prepare_mode(c, mode);
    if (s != DPMT_OK) return s;
    if (mode == DPMT_CP_FP32) {
        ModeData::CpTileSet* cts = nullptr;
        if ((s = prepare_cp_tiles(c, &cts)) != DPMT_OK) return s;
    } else {
        ModeData::TileSet* ts = nullptr;
        if ((s = prepare_tiles(c, mode, &ts)) != DPMT_OK) return s;
    }
    if (!c->aux_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking), "hipStreamCreate");
    while ((int)c->chunk_ev.size() < c->n_chunks + 2) {
        hipEvent_t e = nullptr;
        HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
        c->chunk_ev.push_back(e);
    }
    if (pruning(c, mode) && c->flags_bytes < (size_t)c->resp_elems) {
        HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
        drop_graph(c);
        dfree(c->d_flags);
        c->d_flags = nullptr;
        c->flags_bytes = 0;
        HIP_TRY(c, hipMalloc((void**)&c->d_flags, std::max<size_t>((size_t)c->resp_elems, 16)), "allocate rejection flags");
        c->flags_bytes = (size_t)c->resp_elems;
    }
    ModeData& md = c->modes[mode];
    if (is_tensor(mode)) {
        const size_t need = (size_t)c->n_cells * md.pk.RP * md.pk.esz;
        if (need > c->Z_bytes) {
            HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
            drop_graph(c);
            dfree(c->d_Z);
            c->d_Z = nullptr;
            c->Z_bytes = 0;
            HIP_TRY(c, hipMalloc(&c->d_Z, need), "allocate projected features");
            c->Z_bytes = need;
        }
    }
    return DPMT_OK;
}

ModeData::TileSet& current_tiles(dpmt_ctx* c, dpmt_mode mode) {
    ModeData& md = c->modes[mode];
    const TileCfg& tc = TILE_CFGS[md.tile_cfg];
    return md.tilesets[{tc.ty * (tc.wy / tc.wx), tc.bb, tc.nfb, 32 * tc.wx}];
}

CorrLaunch corr_launch(const ModeData& md) {
    const TileCfg& tc = TILE_CFGS[md.tile_cfg];
    return CorrLaunch{md.kind, md.pk, tc.ty, tc.bb, tc.wy, tc.persistent, tc.wx, 0};
}

// Correlation of the tiles [b, e) of one order of the current tile set
// (0: cost order, 1: (image, level) order, 2: chunk order).
hipError_t corr_tiles(dpmt_ctx* c, dpmt_mode mode, int order, int b, int e, const float* X,
                      hipStream_t st) {
    ModeData& md = c->modes[mode];
    if (mode == DPMT_CP_FP32) {
        ModeData::CpTileSet& ts = md.cp;
        const CpTile* t = order == 0 ? ts.dTiles : order == 1 ? ts.dTilesLvl : ts.dTilesChunk;
        return launch_cp_corr(t + b, e - b, md.dCpChunks, X, md.dCpFac, c->d_resp, c->d_rkeys, c->n_slots,
                              pruning(c, mode) ? c->d_flags : nullptr, ts.lds, st);
    }
    ModeData::TileSet& ts = current_tiles(c, mode);
    const CorrTile* t = order == 0 ? ts.dTiles : order == 1 ? ts.dTilesLvl : ts.dTilesChunk;
    const void* Z = is_tensor(mode) ? c->d_Z : static_cast<const void*>(X);
    // one launch per run of equal filter height: the kernel built for that
    // height alone, with the LDS that height needs
    CorrLaunch cl = corr_launch(md);
    for (const auto& r : ts.runs[order]) {
        const int rb = std::max(b, r[0]), re = std::min(e, r[1]);
        if (rb >= re) continue;
        cl.hs = r[2];
        const hipError_t err = launch_corr(cl, t + rb, re - rb, md.dGroups, Z, md.dG, md.dTk, c->d_resp,
                                           c->d_rkeys, c->n_slots, r[2], r[3], st);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

int n_corr_tiles(dpmt_ctx* c, dpmt_mode mode) {
    return mode == DPMT_CP_FP32 ? c->modes[mode].cp.n_tiles : current_tiles(c, mode).n_tiles;
}
const std::vector<std::array<int, 4>>& corr_levels(dpmt_ctx* c, dpmt_mode mode) {
    return mode == DPMT_CP_FP32 ? c->modes[mode].cp.lvl : current_tiles(c, mode).lvl;
}
const std::vector<std::array<int, 2>>& corr_chunks(dpmt_ctx* c, dpmt_mode mode) {
    return mode == DPMT_CP_FP32 ? c->modes[mode].cp.chunk : current_tiles(c, mode).chunk;
}

// Placement LDS for the maps of n blocks: the tallest map, the tallest and
// widest part map and the most parts among them.
// Dynamic LDS of a placement launch over these blocks: every block lays out
// its own map's buffers, so the launch needs the largest of its maps'.
size_t place_bytes_of(const dpmt_ctx* c, const int2* blk, size_t n) {
    size_t bytes = 0;
    int last = -1;
    for (size_t b = 0; b < n; ++b) {
        if (blk[b].x == last) continue;
        last = blk[b].x;
        bytes = std::max(bytes, place_lds_bytes(place_lds_of_map(c->maps[last])));
    }
    return bytes;
}

// Placement workgroups of 256 threads one CU holds by LDS (at most
// PLACE_WG_PER_CU, the register limit), for a block that needs `bytes` of
// dynamic LDS.
int place_wg_per_cu(size_t bytes) { return place_blocks_per_cu(bytes, 256); }

// The whole call as one launch per stage: value-range reset, projection of
// every level, correlation of every tile, placement of every score map.
hipError_t enqueue_batched(dpmt_ctx* c, dpmt_mode mode, const float* X, float* scores,
                           int16_t* offs, hipStream_t st, hipEvent_t* ev) {
    ModeData& md = c->modes[mode];
    hipError_t e = ev ? hipEventRecord(ev[0], st) : hipSuccess;
    if (e == hipSuccess) {                         // the projection also resets the value ranges
        if (!is_tensor(mode)) e = launch_range_init(c->d_rkeys, c->n_slots, st);
        else if (mode == DPMT_TENSOR_FP8) e = fp8_operands(md, X, c->n_cells, c->d_Z, c->d_rkeys, c->n_slots, st);
        else e = launch_project(md.pk.esz == 2, X, c->n_cells, md.dU, md.pk.RP, c->d_Z, c->d_rkeys, c->n_slots, st);
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = corr_tiles(c, mode, 0, 0, n_corr_tiles(c, mode), X, st);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2], st);
    for (size_t k = 0; k < c->place_runs.size() && e == hipSuccess; ++k)
        e = launch_place(c->d_maps, c->d_parts, c->d_place_blk + c->place_runs[k][0],
                         c->place_runs[k][1] - c->place_runs[k][0], c->d_resp, c->d_rkeys, c->n_slots,
                         scores, offs, c->place_runs_lds[k], pruning(c, mode) ? c->d_flags : nullptr, st);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[3], st);
    return e;
}

// The same work as separate launches per pyramid level: projection and
// correlation of each (image, level), then placement of each (image, root
// level).  FP8 scales stay global, so both strategies compute equal bits.
hipError_t enqueue_per_level(dpmt_ctx* c, dpmt_mode mode, const float* X, float* scores,
                             int16_t* offs, hipStream_t st, hipEvent_t* ev) {
    ModeData& md = c->modes[mode];
    const size_t zcell = (size_t)md.pk.RP * md.pk.esz;
    hipError_t e = ev ? hipEventRecord(ev[0], st) : hipSuccess;
    if (e == hipSuccess) e = launch_range_init(c->d_rkeys, c->n_slots, st);
    if (e == hipSuccess && mode == DPMT_TENSOR_FP8) e = fp8_prepare(md, X, c->n_cells, nullptr, 0, st);
    for (size_t i = 0; i < c->pyr.size() && e == hipSuccess && is_tensor(mode); ++i)
        for (const LevelInfo& lv : c->pyr[i]) {
            if (e != hipSuccess) break;
            const int64_t n = (int64_t)lv.rows * lv.cols;
            const float* Xl = X + lv.cell_offset * 32;
            void* Zl = static_cast<char*>(c->d_Z) + lv.cell_offset * zcell;
            e = mode == DPMT_TENSOR_FP8 ? launch_project_fp8(Xl, n, md.dU, md.pk.RP, md.dScales, Zl, st)
                                        : launch_project(md.pk.esz == 2, Xl, n, md.dU, md.pk.RP, Zl, nullptr, 0, st);
        }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], st);
    for (const auto& r : corr_levels(c, mode)) {
        if (e != hipSuccess) break;
        e = corr_tiles(c, mode, 1, r[2], r[3], X, st);
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2], st);
    for (size_t k = 0; k < c->place_lvl.size() && e == hipSuccess; ++k) {
        const auto& r = c->place_lvl[k];
        e = launch_place(c->d_maps, c->d_parts, c->d_place_blk_lvl + r[2], r[3] - r[2], c->d_resp,
                         c->d_rkeys, c->n_slots, scores, offs, c->place_lvl_lds[k],
                         pruning(c, mode) ? c->d_flags : nullptr, st);
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[3], st);
    return e;
}

// Correlation chunks on the caller's stream; the placement of each chunk on a
// second stream once that chunk's responses are complete, so that placement
// (VALU bound) runs while the next chunks' correlation (MFMA bound) runs.
hipError_t enqueue_overlap(dpmt_ctx* c, dpmt_mode mode, const float* X, float* scores,
                           int16_t* offs, hipStream_t st, hipEvent_t* ev) {
    ModeData& md = c->modes[mode];
    const int K = c->n_chunks;
    hipError_t e = ev ? hipEventRecord(ev[0], st) : hipSuccess;
    if (e == hipSuccess) {                         // the projection also resets the value ranges
        if (!is_tensor(mode)) e = launch_range_init(c->d_rkeys, c->n_slots, st);
        else if (mode == DPMT_TENSOR_FP8) e = fp8_operands(md, X, c->n_cells, c->d_Z, c->d_rkeys, c->n_slots, st);
        else e = launch_project(md.pk.esz == 2, X, c->n_cells, md.dU, md.pk.RP, c->d_Z, c->d_rkeys, c->n_slots, st);
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[1], st);
    hipEvent_t fork = c->chunk_ev[K], join = c->chunk_ev[K + 1];
    if (e == hipSuccess) e = hipEventRecord(fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->aux_stream, fork, 0);
    const auto& chunks = corr_chunks(c, mode);
    for (int k = 0; k < K && e == hipSuccess; ++k) {
        e = corr_tiles(c, mode, 2, chunks[k][0], chunks[k][1], X, st);
        if (e == hipSuccess) e = hipEventRecord(c->chunk_ev[k], st);
        if (e == hipSuccess) e = hipStreamWaitEvent(c->aux_stream, c->chunk_ev[k], 0);
        if (e == hipSuccess)
            e = launch_place(c->d_maps, c->d_parts, c->d_place_blk_chunk + c->place_chunk[k][0],
                             c->place_chunk[k][1] - c->place_chunk[k][0], c->d_resp, c->d_rkeys,
                             c->n_slots, scores, offs, c->place_chunk_lds[k],
                             pruning(c, mode) ? c->d_flags : nullptr, c->aux_stream);
    }
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2], st);
    if (e == hipSuccess) e = hipEventRecord(join, c->aux_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, join, 0);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[3], st);
    return e;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* dpmt_status_string(dpmt_status s) {
    switch (s) {
        case DPMT_OK: return "ok";
        case DPMT_E_INVALID: return "invalid argument";
        case DPMT_E_STATE: return "call out of order";
        case DPMT_E_RANK: return "rank outside [1, 32]";
        case DPMT_E_NOMEM: return "out of memory";
        case DPMT_E_DEVICE: return "device error";
        case DPMT_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* dpmt_last_error(const dpmt_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_free_error.c_str();
}

dpmt_status dpmt_create(dpmt_ctx** out, int32_t device, void* hip_stream) {
    if (!out) return fail(nullptr, DPMT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (device < -1) return fail(nullptr, DPMT_E_INVALID, "device must be >= -1");
    dpmt_ctx* c = new dpmt_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || device >= n) {
            delete c;
            return fail(nullptr, DPMT_E_DEVICE, "no such HIP device");
        }
        e = hipSetDevice(device);
        if (e != hipSuccess) {
            delete c;
            return fail(nullptr, DPMT_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
        }
    }
    *out = c;
    return DPMT_OK;
}

void dpmt_destroy(dpmt_ctx* c) {
    if (!c) return;
    if (c->has_device()) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        free_plan(c);
        for (auto& m : c->modes) free_mode(m);
        dfree(c->d_hog_levels);
        dfree(c->d_hog_tiles);
        dfree(c->d_hog_blocks);
        dfree(c->d_hog_hist);
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
        for (hipEvent_t e : c->chunk_ev) (void)hipEventDestroy(e);
        for (auto& set : c->ev_sets)
            for (auto& e : set) (void)hipEventDestroy(e);
    }
    delete c;
}

dpmt_status dpmt_load_filters(dpmt_ctx* c, int32_t n_filters, const dpmt_shape* shapes,
                              const float* weights_host, int32_t n_components,
                              const dpmt_component* comps) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (n_filters <= 0 || !shapes || !weights_host) return fail(c, DPMT_E_INVALID, "need n_filters > 0, shapes and weights");
    if (n_components <= 0 || !comps) return fail(c, DPMT_E_INVALID, "need n_components > 0 and comps");
    int64_t total = 0;
    for (int k = 0; k < n_filters; ++k) {
        if (shapes[k].h < 1 || shapes[k].w < 1) return fail(c, DPMT_E_INVALID, "filter " + std::to_string(k) + " has an empty shape");
        if (shapes[k].h > MAX_FILTER_H || shapes[k].w > MAX_FILTER_W)
            return fail(c, DPMT_E_UNSUPPORTED, "filter " + std::to_string(k) + " larger than 16 x 32 cells");
        total += (int64_t)shapes[k].h * shapes[k].w * 32;
    }
    for (int64_t i = 0; i < total; ++i)
        if (!std::isfinite(weights_host[i])) return fail(c, DPMT_E_INVALID, "non-finite filter weight at element " + std::to_string(i));
    for (int ci = 0; ci < n_components; ++ci) {
        const dpmt_component& cm = comps[ci];
        const std::string cs = "component " + std::to_string(ci) + ": ";
        if (cm.root < 0 || cm.root >= n_filters) return fail(c, DPMT_E_INVALID, cs + "root index out of range");
        if (cm.n_parts < 1 || !cm.parts || !cm.anchors || !cm.deform) return fail(c, DPMT_E_INVALID, cs + "needs n_parts >= 1 with parts, anchors, deform");
        if (cm.n_parts > 64) return fail(c, DPMT_E_UNSUPPORTED, cs + "more than 64 parts");
        const int h0 = shapes[cm.root].h, w0 = shapes[cm.root].w;
        for (int i = 0; i < cm.n_parts; ++i) {
            const int k = cm.parts[i];
            if (k < 0 || k >= n_filters) return fail(c, DPMT_E_INVALID, cs + "part index out of range");
            const float* d = cm.deform + 4 * i;
            for (int t = 0; t < 4; ++t)
                if (!std::isfinite(d[t])) return fail(c, DPMT_E_INVALID, cs + "non-finite deformation coefficient");
            if (!(d[1] > 0.f) || !(d[3] > 0.f)) return fail(c, DPMT_E_INVALID, cs + "quadratic deformation coefficients must be > 0");
            const int vy = cm.anchors[2 * i], vx = cm.anchors[2 * i + 1];
            if (vy < 0 || vx < 0 || vy > 2 * h0 - shapes[k].h || vx > 2 * w0 - shapes[k].w)
                return fail(c, DPMT_E_INVALID, cs + "anchor of part " + std::to_string(i) + " outside [0, 2*h0-h] x [0, 2*w0-w]");
        }
    }
    // accepted: replace the bank
    if (c->has_device()) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        free_plan(c);
        for (auto& m : c->modes) free_mode(m);
    }
    for (auto& m : c->modes) m.tile_cfg = 0;
    c->planned = false;
    c->decomposed = false;
    c->cp_ready = false;
    c->cp_rank.clear();
    c->cp_off.clear();
    c->cp_fac.clear();
    c->thr_set = false;
    c->cp_thr.clear();
    c->thr_off.clear();
    c->shapes.assign(shapes, shapes + n_filters);
    c->woff.resize(n_filters);
    int64_t off = 0;
    for (int k = 0; k < n_filters; ++k) {
        c->woff[k] = off;
        off += (int64_t)shapes[k].h * shapes[k].w * 32;
    }
    c->weights.assign(weights_host, weights_host + total);
    c->comps.clear();
    for (int ci = 0; ci < n_components; ++ci) {
        const dpmt_component& cm = comps[ci];
        dpmt_ctx::Comp cp;
        cp.root = cm.root;
        for (int i = 0; i < cm.n_parts; ++i) {
            cp.parts.push_back(cm.parts[i]);
            cp.anchors.push_back({cm.anchors[2 * i], cm.anchors[2 * i + 1]});
            cp.deform.push_back({cm.deform[4 * i], cm.deform[4 * i + 1], cm.deform[4 * i + 2], cm.deform[4 * i + 3]});
        }
        c->comps.push_back(cp);
    }
    build_groups(c);
    c->loaded = true;
    c->err.clear();
    return DPMT_OK;
}

dpmt_status dpmt_decompose(dpmt_ctx* c, int32_t rank, double* sigma_out, double* basis_out) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (!c->loaded) return fail(c, DPMT_E_STATE, "dpmt_decompose before dpmt_load_filters");
    if (rank < 1 || rank > 32) return fail(c, DPMT_E_RANK, "rank must be in [1, 32]");
    // Gram matrix of the mode-3 unfolding: sum over every filter cell of v v^T
    std::vector<double> C(32 * 32, 0.0);
    const int64_t n_cells = (int64_t)c->weights.size() / 32;
    for (int64_t i = 0; i < n_cells; ++i) {
        const float* v = c->weights.data() + i * 32;
        for (int a = 0; a < 32; ++a) {
            const double va = v[a];
            for (int b = 0; b < 32; ++b) C[a * 32 + b] += va * (double)v[b];
        }
    }
    std::vector<double> V;
    jacobi_eigen(C, V, 32);
    std::vector<int> order(32);
    for (int i = 0; i < 32; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return C[a * 32 + a] > C[b * 32 + b]; });
    c->sigma.assign(32, 0.0);
    c->Ufull.assign(32 * 32, 0.0);
    for (int j = 0; j < 32; ++j) {
        const int src = order[j];
        c->sigma[j] = std::sqrt(std::max(C[src * 32 + src], 0.0));
        int imax = 0;
        for (int l = 1; l < 32; ++l)
            if (std::fabs(V[l * 32 + src]) > std::fabs(V[imax * 32 + src])) imax = l;
        const double sg = V[imax * 32 + src] < 0 ? -1.0 : 1.0;
        for (int l = 0; l < 32; ++l) c->Ufull[l * 32 + j] = sg * V[l * 32 + src];
    }
    c->rank = rank;
    c->decomposed = true;
    if (c->has_device()) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
    }
    drop_graph(c);
    for (int m = 1; m < 4; ++m) free_mode(c->modes[m]);   // tensor operands depend on U_R
    if (sigma_out) std::memcpy(sigma_out, c->sigma.data(), 32 * sizeof(double));
    if (basis_out)
        for (int l = 0; l < 32; ++l)
            for (int r = 0; r < rank; ++r) basis_out[l * rank + r] = c->Ufull[l * 32 + r];
    if (c->has_device()) {
        // upload the factors of the modes the build supports now, so that the
        // first score call does not pay for packing
        dpmt_status s = prepare_mode(c, DPMT_TENSOR_BF16);
        if (s != DPMT_OK) return s;
    }
    c->err.clear();
    return DPMT_OK;
}

namespace {
// Replace the CP factors and drop what was built from the previous ones.
void set_cp(dpmt_ctx* c, std::vector<int> rank, std::vector<int64_t> off, std::vector<float> fac) {
    if (c->has_device()) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
    }
    drop_graph(c);
    free_mode(c->modes[DPMT_CP_FP32]);
    c->cp_rank = std::move(rank);
    c->cp_off = std::move(off);
    c->cp_fac = std::move(fac);
    c->cp_ready = true;
    c->thr_set = false;
    c->cp_thr.clear();
    c->thr_off.clear();
}

dpmt_status cp_ranks_check(dpmt_ctx* c, const int32_t* ranks, std::vector<int64_t>& off, int64_t& total) {
    if (!ranks) return fail(c, DPMT_E_INVALID, "ranks is NULL");
    off.assign(c->shapes.size(), 0);
    total = 0;
    for (size_t k = 0; k < c->shapes.size(); ++k) {
        if (ranks[k] < 1 || ranks[k] > 32) return fail(c, DPMT_E_RANK, "rank of filter " + std::to_string(k) + " outside [1, 32]");
        off[k] = total;
        total += (int64_t)ranks[k] * (c->shapes[k].h + c->shapes[k].w + 32);
    }
    return DPMT_OK;
}
}  // namespace

dpmt_status dpmt_decompose_cp(dpmt_ctx* c, const int32_t* ranks, int32_t max_iters, double tol,
                              double* rel_err_out) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (!c->loaded) return fail(c, DPMT_E_STATE, "dpmt_decompose_cp before dpmt_load_filters");
    if (max_iters < 1) return fail(c, DPMT_E_INVALID, "max_iters must be >= 1");
    if (!(tol >= 0) || !std::isfinite(tol)) return fail(c, DPMT_E_INVALID, "tol must be finite and >= 0");
    std::vector<int64_t> off;
    int64_t total = 0;
    dpmt_status s = cp_ranks_check(c, ranks, off, total);
    if (s != DPMT_OK) return s;
    const int nf = (int)c->shapes.size();
    std::vector<float> fac((size_t)total);
    std::vector<double> err(nf);
    // filters are independent: fitted on up to 16 host threads
    const int nt = std::max(1, std::min<int>({16, nf, (int)std::max(1u, std::thread::hardware_concurrency())}));
    auto work = [&](int t0) {
        for (int k = t0; k < nf; k += nt) {
            const int h = c->shapes[k].h, w = c->shapes[k].w, R = ranks[k];
            const CpFit fit = cp_als(c->weights.data() + c->woff[k], h, w, 32, R, max_iters, tol);
            float* dst = fac.data() + off[k];
            for (size_t i = 0; i < fit.A.size(); ++i) dst[i] = (float)fit.A[i];
            dst += fit.A.size();
            for (size_t i = 0; i < fit.B.size(); ++i) dst[i] = (float)fit.B[i];
            dst += fit.B.size();
            for (size_t i = 0; i < fit.C.size(); ++i) dst[i] = (float)fit.C[i];
            err[k] = fit.rel_err;
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto& th : pool) th.join();
    set_cp(c, std::vector<int>(ranks, ranks + nf), std::move(off), std::move(fac));
    if (rel_err_out) std::memcpy(rel_err_out, err.data(), nf * sizeof(double));
    c->err.clear();
    return DPMT_OK;
}

dpmt_status dpmt_select_ranks(dpmt_ctx* c, double e, int32_t r_max, int32_t max_iters,
                              int32_t* ranks_out, double* rel_err_out) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (!c->loaded) return fail(c, DPMT_E_STATE, "dpmt_select_ranks before dpmt_load_filters");
    if (!(e >= 0) || !std::isfinite(e)) return fail(c, DPMT_E_INVALID, "e must be finite and >= 0");
    if (r_max < 1 || r_max > 32) return fail(c, DPMT_E_RANK, "r_max must be in [1, 32]");
    if (max_iters < 1) return fail(c, DPMT_E_INVALID, "max_iters must be >= 1");
    const int nf = (int)c->shapes.size();
    std::vector<int> rank(nf, 1);
    std::vector<CpFit> chosen(nf);
    const int nt = std::max(1, std::min<int>({16, nf, (int)std::max(1u, std::thread::hardware_concurrency())}));
    auto work = [&](int t0) {
        for (int k = t0; k < nf; k += nt) {
            const int h = c->shapes[k].h, w = c->shapes[k].w;
            const float* f = c->weights.data() + c->woff[k];
            double nrm = 0;
            for (int i = 0; i < h * w * 32; ++i) nrm += (double)f[i] * f[i];
            nrm = std::sqrt(nrm);
            std::map<int, CpFit> fits;
            auto ok = [&](int r) {
                auto it = fits.find(r);
                if (it == fits.end()) it = fits.emplace(r, cp_als(f, h, w, 32, r, max_iters, 1e-13)).first;
                const double g = (double)r * (h + w + 32) / ((double)h * w * 32);
                return it->second.rel_err * nrm < e * g * g;       // Section 4 rank criterion
            };
            int lo = 1, hi = r_max;
            while (lo < hi) {
                const int mid = (lo + hi) / 2;
                if (ok(mid)) hi = mid;
                else lo = mid + 1;
            }
            if (!fits.count(lo)) fits.emplace(lo, cp_als(f, h, w, 32, lo, max_iters, 1e-13));
            rank[k] = lo;
            chosen[k] = std::move(fits[lo]);
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto& th : pool) th.join();
    std::vector<int64_t> off(nf);
    int64_t total = 0;
    for (int k = 0; k < nf; ++k) {
        off[k] = total;
        total += (int64_t)rank[k] * (c->shapes[k].h + c->shapes[k].w + 32);
    }
    std::vector<float> fac((size_t)total);
    for (int k = 0; k < nf; ++k) {
        float* dst = fac.data() + off[k];
        for (double v : chosen[k].A) *dst++ = (float)v;
        for (double v : chosen[k].B) *dst++ = (float)v;
        for (double v : chosen[k].C) *dst++ = (float)v;
        if (ranks_out) ranks_out[k] = rank[k];
        if (rel_err_out) rel_err_out[k] = chosen[k].rel_err;
    }
    set_cp(c, std::move(rank), std::move(off), std::move(fac));
    c->err.clear();
    return DPMT_OK;
}

namespace {
// Replace the thresholds (empty: none) and drop what was packed with the old ones.
void set_thresholds(dpmt_ctx* c, std::vector<float> t) {
    if (c->has_device()) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
    }
    drop_graph(c);
    free_mode(c->modes[DPMT_CP_FP32]);
    c->thr_set = !t.empty();
    c->cp_thr = std::move(t);
    c->thr_off.assign(c->shapes.size(), 0);
    int64_t o = 0;
    for (size_t k = 0; k < c->shapes.size(); ++k) {
        c->thr_off[k] = o;
        o += c->cp_rank[k];
    }
}

// Partial sums p_r (r = 1..R) of filter k's CP terms at (y, x) of a level
// (FP64 over the stored FP32 factors): term r = sum_n a_r[n] sum_m b_r[m]
// (X[y+n][x+m] . c_r).
void cp_partials(const dpmt_ctx* c, int k, const float* X, int cols, int y, int x, std::vector<double>& p) {
    const int h = c->shapes[k].h, w = c->shapes[k].w, R = c->cp_rank[k];
    const float* A = c->cp_fac.data() + c->cp_off[k];
    const float* B = A + (int64_t)h * R;
    const float* C = B + (int64_t)w * R;
    p.assign(R, 0.0);
    double run = 0;
    for (int r = 0; r < R; ++r) {
        double term = 0;
        for (int n = 0; n < h; ++n) {
            double row = 0;
            for (int m = 0; m < w; ++m) {
                const float* cell = X + ((int64_t)(y + n) * cols + (x + m)) * 32;
                double z = 0;
                for (int l = 0; l < 32; ++l) z += (double)cell[l] * C[l * R + r];
                row += (double)B[m * R + r] * z;
            }
            term += (double)A[n * R + r] * row;
        }
        run += term;
        p[r] = run;
    }
}
}  // namespace

dpmt_status dpmt_set_thresholds(dpmt_ctx* c, const float* thresholds_host) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (!c->cp_ready) return fail(c, DPMT_E_STATE, "thresholds need CP factors first");
    if (!thresholds_host) {
        set_thresholds(c, {});
        return DPMT_OK;
    }
    int64_t n = 0;
    for (int r : c->cp_rank) n += r;
    for (int64_t i = 0; i < n; ++i)
        if (std::isnan(thresholds_host[i])) return fail(c, DPMT_E_INVALID, "NaN threshold at element " + std::to_string(i));
    set_thresholds(c, std::vector<float>(thresholds_host, thresholds_host + n));
    c->err.clear();
    return DPMT_OK;
}

dpmt_status dpmt_fit_thresholds(dpmt_ctx* c, const float* features_host, int32_t n_pos,
                                const dpmt_hypothesis* pos, float margin, float* thresholds_out) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (!c->cp_ready) return fail(c, DPMT_E_STATE, "thresholds need CP factors first");
    if (!c->planned) return fail(c, DPMT_E_STATE, "dpmt_fit_thresholds before dpmt_plan");
    if (!features_host || !pos || n_pos < 1) return fail(c, DPMT_E_INVALID, "need features_host and n_pos >= 1 positives");
    if (!std::isfinite(margin) || margin < 0) return fail(c, DPMT_E_INVALID, "margin must be finite and >= 0");
    for (int i = 0; i < n_pos; ++i) {
        const dpmt_hypothesis& g = pos[i];
        const std::string ps = "positive " + std::to_string(i) + ": ";
        if (g.image < 0 || g.image >= (int)c->pyr.size()) return fail(c, DPMT_E_INVALID, ps + "image out of range");
        const int oct = c->octave[g.image];
        if (g.level < oct || g.level >= (int)c->pyr[g.image].size()) return fail(c, DPMT_E_INVALID, ps + "not a root level");
        if (g.comp < 0 || g.comp >= (int)c->comps.size()) return fail(c, DPMT_E_INVALID, ps + "component out of range");
        const LevelInfo& lv = c->pyr[g.image][g.level];
        const dpmt_shape& r0 = c->shapes[c->comps[g.comp].root];
        if (g.y < 0 || g.x < 0 || g.y > lv.rows - r0.h || g.x > lv.cols - r0.w)
            return fail(c, DPMT_E_INVALID, ps + "position outside the score map");
    }
    const int nf = (int)c->shapes.size();
    std::vector<std::vector<double>> lo(nf);
    std::vector<double> p;
    auto take = [&](int k, const LevelInfo& lv, int y, int x) {
        cp_partials(c, k, features_host + lv.cell_offset * 32, lv.cols, y, x, p);
        if (lo[k].empty()) lo[k] = p;
        else
            for (size_t r = 0; r < p.size(); ++r) lo[k][r] = std::min(lo[k][r], p[r]);
    };
    for (int i = 0; i < n_pos; ++i) {
        const dpmt_hypothesis& g = pos[i];
        const dpmt_ctx::Comp& cm = c->comps[g.comp];
        take(cm.root, c->pyr[g.image][g.level], g.y, g.x);
        const LevelInfo& pl = c->pyr[g.image][g.level - c->octave[g.image]];
        for (size_t s = 0; s < cm.parts.size(); ++s) {
            const int k = cm.parts[s];
            const int ay = 2 * g.y + cm.anchors[s][0], ax = 2 * g.x + cm.anchors[s][1];
            if (ay <= pl.rows - c->shapes[k].h && ax <= pl.cols - c->shapes[k].w) take(k, pl, ay, ax);
        }
    }
    std::vector<float> t;
    for (int k = 0; k < nf; ++k)
        for (int r = 0; r < c->cp_rank[k]; ++r)
            t.push_back(lo[k].empty() ? -INFINITY : (float)(lo[k][r] - (double)margin));
    if (thresholds_out) std::memcpy(thresholds_out, t.data(), t.size() * sizeof(float));
    set_thresholds(c, std::move(t));
    c->err.clear();
    return DPMT_OK;
}

dpmt_status dpmt_load_cp(dpmt_ctx* c, const int32_t* ranks, const float* factors_host) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (!c->loaded) return fail(c, DPMT_E_STATE, "dpmt_load_cp before dpmt_load_filters");
    std::vector<int64_t> off;
    int64_t total = 0;
    dpmt_status s = cp_ranks_check(c, ranks, off, total);
    if (s != DPMT_OK) return s;
    if (!factors_host) return fail(c, DPMT_E_INVALID, "factors_host is NULL");
    for (int64_t i = 0; i < total; ++i)
        if (!std::isfinite(factors_host[i])) return fail(c, DPMT_E_INVALID, "non-finite CP factor at element " + std::to_string(i));
    set_cp(c, std::vector<int>(ranks, ranks + c->shapes.size()), std::move(off),
           std::vector<float>(factors_host, factors_host + total));
    c->err.clear();
    return DPMT_OK;
}

dpmt_status dpmt_get_cp(const dpmt_ctx* c, int32_t* ranks_out, float* factors_out, int64_t* n_floats) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (!c->cp_ready) return fail(const_cast<dpmt_ctx*>(c), DPMT_E_STATE, "no CP factors");
    if (n_floats) *n_floats = (int64_t)c->cp_fac.size();
    if (ranks_out)
        for (size_t k = 0; k < c->cp_rank.size(); ++k) ranks_out[k] = c->cp_rank[k];
    if (factors_out) std::memcpy(factors_out, c->cp_fac.data(), c->cp_fac.size() * sizeof(float));
    return DPMT_OK;
}

dpmt_status dpmt_plan(dpmt_ctx* c, int32_t n_images, const dpmt_pyramid* pyrs, const dpmt_layout** out) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (!c->loaded) return fail(c, DPMT_E_STATE, "dpmt_plan before dpmt_load_filters");
    if (n_images <= 0 || !pyrs || !out) return fail(c, DPMT_E_INVALID, "need n_images > 0, pyrs and out");
    for (int i = 0; i < n_images; ++i) {
        const dpmt_pyramid& p = pyrs[i];
        if (p.n_levels < 1 || !p.levels) return fail(c, DPMT_E_INVALID, "image " + std::to_string(i) + ": empty pyramid");
        if (p.octave < 1) return fail(c, DPMT_E_INVALID, "image " + std::to_string(i) + ": octave must be >= 1");
        for (int l = 0; l < p.n_levels; ++l) {
            const dpmt_level& lv = p.levels[l];
            if (lv.rows < 1 || lv.cols < 1 || lv.cell_offset < 0)
                return fail(c, DPMT_E_INVALID, "image " + std::to_string(i) + " level " + std::to_string(l) + ": bad size or offset");
            if ((int64_t)lv.rows * lv.cols > (int64_t)1 << 30)
                return fail(c, DPMT_E_UNSUPPORTED, "level larger than 2^30 cells");
            if (lv.rows > 16384 || lv.cols > 16384)
                return fail(c, DPMT_E_UNSUPPORTED, "level side longer than 16384 cells");
        }
    }
    if (c->has_device()) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
    }
    free_plan(c);
    c->plan_id++;
    c->pyr.assign(n_images, {});
    c->octave.assign(n_images, 0);
    c->n_cells = 0;
    for (int i = 0; i < n_images; ++i) {
        c->octave[i] = pyrs[i].octave;
        for (int l = 0; l < pyrs[i].n_levels; ++l) {
            const dpmt_level& lv = pyrs[i].levels[l];
            c->pyr[i].push_back(LevelInfo{lv.cell_offset, lv.rows, lv.cols});
            c->n_cells = std::max(c->n_cells, lv.cell_offset + (int64_t)lv.rows * lv.cols);
        }
    }
    // response blocks: root groups on levels >= octave, part groups one octave
    // below; one plane per filter with a pitch of whole 16-byte runs
    c->blocks.clear();
    c->resp_elems = 0;
    c->n_slots = 0;
    int64_t n_root = 0, n_part = 0;
    for (int i = 0; i < n_images; ++i) {
        const int L = (int)c->pyr[i].size(), oct = c->octave[i];
        for (size_t g = 0; g < c->groups.size(); ++g) {
            const HostGroup& hg = c->groups[g];
            if (hg.role == ROLE_ALL) continue;
            const int l_lo = hg.role == ROLE_ROOT ? oct : 0;
            const int l_hi = hg.role == ROLE_ROOT ? L : L - oct;
            for (int l = l_lo; l < l_hi; ++l) {
                const LevelInfo& lv = c->pyr[i][l];
                const int Ho = lv.rows - hg.h + 1, Wo = lv.cols - hg.w + 1;
                if (Ho <= 0 || Wo <= 0) continue;
                const int ld = pitch_of(Wo);
                c->blocks[BlockKey{i, l, (int)g}] = BlockInfo{c->resp_elems, Ho, Wo, ld, c->n_slots};
                const int64_t ng = (int64_t)hg.filters.size();
                c->resp_elems += ng * Ho * ld;
                c->n_slots += ng;
                (hg.role == ROLE_ROOT ? n_root : n_part) += ng * Ho * Wo;
            }
        }
    }
    if (c->n_slots >= INT32_MAX) return fail(c, DPMT_E_UNSUPPORTED, "batch has too many response planes");
    // score maps and their parts
    c->m_image.clear(); c->m_level.clear(); c->m_comp.clear(); c->m_rows.clear(); c->m_cols.clear();
    c->m_score_off.clear(); c->m_offs_off.clear(); c->maps.clear(); c->map_parts.clear();
    int64_t score_off = 0, offs_off = 0;
    int max_Wp = 0;
    for (int i = 0; i < n_images; ++i) {
        const int L = (int)c->pyr[i].size(), oct = c->octave[i];
        for (int l = oct; l < L; ++l) {
            const LevelInfo& lv = c->pyr[i][l];
            for (size_t ci = 0; ci < c->comps.size(); ++ci) {
                const auto& cm = c->comps[ci];
                const dpmt_shape rs = c->shapes[cm.root];
                const int Ho = std::max(lv.rows - rs.h + 1, 0), Wo = std::max(lv.cols - rs.w + 1, 0);
                const int np = (int)cm.parts.size();
                MapDesc md{};
                int map_Hp = 0, map_Wp = 0;               // tallest and widest part map
                md.score_off = score_off;
                md.offs_off = offs_off;
                md.Ho = Ho;
                md.Wo = Wo;
                md.n_parts = np;
                md.part_base = (int)c->map_parts.size();
                auto rb = c->blocks.find(BlockKey{i, l, c->comp_root_group[ci]});
                if (rb != c->blocks.end()) {
                    md.root_plane = rb->second.off + (int64_t)c->comp_root_col[ci] * rb->second.Ho * rb->second.ld;
                    md.ldr = rb->second.ld;
                }
                for (int sl = 0; sl < np; ++sl) {
                    MapPart mp{};
                    const auto gc = c->comp_part_gc[ci][sl];
                    auto pb = c->blocks.find(BlockKey{i, l - oct, gc.first});
                    if (pb != c->blocks.end()) {
                        const BlockInfo& bi = pb->second;
                        mp.plane = bi.off + (int64_t)gc.second * bi.Ho * bi.ld;
                        mp.ld = bi.ld;
                        mp.Hp = bi.Ho;
                        mp.Wp = bi.Wo;
                        mp.rng = (int32_t)(bi.rng + gc.second);
                    }
                    mp.vy = cm.anchors[sl][0];
                    mp.vx = cm.anchors[sl][1];
                    for (int t = 0; t < 4; ++t) mp.d[t] = cm.deform[sl][t];
                    mp.inv2ax = (float)(0.5 / (double)mp.d[1]);
                    mp.inv2ay = (float)(0.5 / (double)mp.d[3]);
                    mp.bb4a = (float)((double)mp.d[0] * mp.d[0] / (4.0 * mp.d[1]));
                    if (Ho > 0 && Wo > 0) max_Wp = std::max(max_Wp, mp.Wp);
                    map_Hp = std::max(map_Hp, mp.Hp);
                    map_Wp = std::max(map_Wp, mp.Wp);
                    c->map_parts.push_back(mp);
                }
                md.r1_rows = map_Hp + 2 * PLACE_PAD;
                md.ctab_words = place_ctab_words(map_Hp, map_Wp);
                c->maps.push_back(md);
                c->m_image.push_back(i);
                c->m_level.push_back(l);
                c->m_comp.push_back((int)ci);
                c->m_rows.push_back(Ho);
                c->m_cols.push_back(Wo);
                c->m_score_off.push_back(score_off);
                c->m_offs_off.push_back(offs_off);
                const int64_t plane = (int64_t)Ho * Wo;
                score_off += plane;
                offs_off += plane * np * 2;
            }
        }
    }
    if (c->map_parts.size() >= (size_t)INT32_MAX) return fail(c, DPMT_E_UNSUPPORTED, "batch has too many score maps");
    // placement blocks: (map, strip of PLACE_CW root columns), largest work first
    // so that the launch ends on short blocks
    {
        std::vector<std::pair<int64_t, int>> order;
        for (size_t k = 0; k < c->maps.size(); ++k) {
            const MapDesc& md = c->maps[k];
            if (md.Ho <= 0 || md.Wo <= 0) continue;
            int64_t work = 0;
            for (int sl = 0; sl < md.n_parts; ++sl) work += c->map_parts[md.part_base + sl].Hp + md.Ho;
            order.push_back({-work, (int)k});
        }
        std::stable_sort(order.begin(), order.end());
        c->place_blk.clear();
        int64_t nb = 0;
        for (const auto& o : order) nb += (c->maps[o.second].Wo + PLACE_CW - 1) / PLACE_CW;
        if (nb > INT32_MAX) return fail(c, DPMT_E_UNSUPPORTED, "batch too large for one launch");
        for (const auto& o : order) {
            const int strips = (c->maps[o.second].Wo + PLACE_CW - 1) / PLACE_CW;
            for (int st = 0; st < strips; ++st) c->place_blk.push_back(make_int2(o.second, st));
        }
        // the same blocks grouped by (image, root level) for per-level launches
        c->place_blk_lvl.clear();
        c->place_lvl.clear();
        for (size_t k = 0; k < c->maps.size(); ++k) {
            const MapDesc& md = c->maps[k];
            if (md.Ho <= 0 || md.Wo <= 0) continue;
            const int img = c->m_image[k], lvl = c->m_level[k];
            const int b0 = (int)c->place_blk_lvl.size();
            for (int st = 0; st < (md.Wo + PLACE_CW - 1) / PLACE_CW; ++st)
                c->place_blk_lvl.push_back(make_int2((int)k, st));
            if (!c->place_lvl.empty() && c->place_lvl.back()[0] == img && c->place_lvl.back()[1] == lvl)
                c->place_lvl.back()[3] = (int)c->place_blk_lvl.size();
            else
                c->place_lvl.push_back({img, lvl, b0, (int)c->place_blk_lvl.size()});
        }
        // dependency groups (image, root level): the responses of root level l
        // and of its part level l - octave, and the score maps of level l.
        // Cheapest first, cut into chunks of about equal response count.
        {
            std::map<std::pair<int, int>, int64_t> work;
            for (size_t k = 0; k < c->maps.size(); ++k) work[{c->m_image[k], c->m_level[k]}] += 0;
            for (const auto& kv : c->blocks) {
                const HostGroup& hg = c->groups[kv.first.group];
                const int lvl = hg.role == ROLE_ROOT ? kv.first.level : kv.first.level + c->octave[kv.first.img];
                work[{kv.first.img, lvl}] += (int64_t)kv.second.Ho * kv.second.Wo * (int64_t)hg.filters.size();
            }
            std::vector<std::pair<int64_t, std::pair<int, int>>> order;
            int64_t total_work = 0;
            for (const auto& kv : work) {
                order.push_back({kv.second, kv.first});
                total_work += kv.second;
            }
            std::stable_sort(order.begin(), order.end());
            const int K = (int)std::min<size_t>(PLACE_CHUNKS, std::max<size_t>(order.size(), 1));
            c->chunk_of.clear();
            int64_t acc_work = 0;
            for (const auto& o : order) {
                const int k = total_work > 0 ? (int)std::min<int64_t>(K - 1, acc_work * K / total_work) : 0;
                c->chunk_of[o.second] = k;
                acc_work += o.first;
            }
            c->n_chunks = K;
            c->place_blk_chunk.clear();
            c->place_chunk.assign(K, {0, 0});
            std::vector<std::vector<int2>> per(K);
            for (const int2& b : c->place_blk) {            // keeps the work order within a chunk
                const int k = c->chunk_of[{c->m_image[b.x], c->m_level[b.x]}];
                per[k].push_back(b);
            }
            for (int k = 0; k < K; ++k) {
                c->place_chunk[k][0] = (int)c->place_blk_chunk.size();
                c->place_blk_chunk.insert(c->place_blk_chunk.end(), per[k].begin(), per[k].end());
                c->place_chunk[k][1] = (int)c->place_blk_chunk.size();
            }
        }
        const int span = place_span_max(max_Wp);
        if (span > PLACE_STAGE)
            return fail(c, DPMT_E_UNSUPPORTED, "part level wider than the placement staging supports");
        if (place_bytes_of(c, c->place_blk.data(), c->place_blk.size()) > PLACE_LDS_MAX)
            return fail(c, DPMT_E_UNSUPPORTED, "score maps too tall for one placement block");
        // batched launch: blocks regrouped (stably, so largest work first
        // within a run) into runs of equal workgroups per CU, fewest first;
        // each run's LDS sized by its own maps, so that short maps are not
        // held to the occupancy of the tallest
        {
            std::vector<std::pair<int, int2>> cls;
            cls.reserve(c->place_blk.size());
            std::map<int, int> wg_of;                     // map -> workgroups per CU
            for (const int2& b : c->place_blk) {
                auto it = wg_of.find(b.x);
                if (it == wg_of.end())
                    it = wg_of.emplace(b.x, place_wg_per_cu(place_lds_bytes(place_lds_of_map(c->maps[b.x])))).first;
                cls.push_back({it->second, b});
            }
            std::stable_sort(cls.begin(), cls.end(),
                             [](const std::pair<int, int2>& a, const std::pair<int, int2>& b) { return a.first < b.first; });
            c->place_runs.clear();
            c->place_runs_lds.clear();
            for (size_t b = 0; b < cls.size(); ++b) {
                c->place_blk[b] = cls[b].second;
                if (b == 0 || cls[b].first != cls[b - 1].first) c->place_runs.push_back({(int)b, (int)b + 1});
                else c->place_runs.back()[1] = (int)b + 1;
            }
            for (const auto& r : c->place_runs)
                c->place_runs_lds.push_back(place_bytes_of(c, c->place_blk.data() + r[0], (size_t)(r[1] - r[0])));
            c->place_lvl_lds.clear();
            for (const auto& r : c->place_lvl)
                c->place_lvl_lds.push_back(place_bytes_of(c, c->place_blk_lvl.data() + r[2], (size_t)(r[3] - r[2])));
            c->place_chunk_lds.clear();
            for (const auto& r : c->place_chunk)
                c->place_chunk_lds.push_back(place_bytes_of(c, c->place_blk_chunk.data() + r[0], (size_t)(r[1] - r[0])));
        }
    }

    dpmt_layout& lay = c->layout;
    lay = dpmt_layout{};
    lay.n_score = score_off;
    lay.n_offsets = offs_off;
    lay.n_maps = (int32_t)c->maps.size();
    lay.map_image = c->m_image.data();
    lay.map_level = c->m_level.data();
    lay.map_comp = c->m_comp.data();
    lay.map_rows = c->m_rows.data();
    lay.map_cols = c->m_cols.data();
    lay.map_score_off = c->m_score_off.data();
    lay.map_offs_off = c->m_offs_off.data();
    lay.n_cells = c->n_cells;
    lay.n_resp = n_root + n_part;
    lay.n_resp_root = n_root;
    lay.n_resp_part = n_part;
    lay.workspace_bytes = c->resp_elems * 4 + c->n_slots * 8 + (det_blocks(score_off) + 1) * 8;

    if (c->has_device()) {
        auto alloc = [&](void** p, int64_t bytes, const char* what) -> dpmt_status {
            if (bytes <= 0) return DPMT_OK;
            hipError_t e = hipMalloc(p, (size_t)bytes);
            if (e != hipSuccess) return hip_fail(c, e, what);
            return DPMT_OK;
        };
        dpmt_status s;
        if ((s = alloc((void**)&c->d_resp, c->resp_elems * 4, "allocate responses")) != DPMT_OK) return s;
        if ((s = alloc((void**)&c->d_rkeys, std::max<int64_t>(c->n_slots, 1) * 8, "allocate value ranges")) != DPMT_OK) return s;
        HIP_TRY(c, upload(&c->d_maps, c->maps), "upload maps");
        HIP_TRY(c, upload(&c->d_parts, c->map_parts), "upload map parts");
        HIP_TRY(c, upload(&c->d_place_blk, c->place_blk), "upload block map");
        HIP_TRY(c, upload(&c->d_place_blk_lvl, c->place_blk_lvl), "upload block map");
        HIP_TRY(c, upload(&c->d_place_blk_chunk, c->place_blk_chunk), "upload block map");
        if ((s = alloc((void**)&c->d_det_counts, (det_blocks(score_off) + 1) * 8, "allocate detection scratch")) != DPMT_OK) return s;
    }
    c->planned = true;
    *out = &c->layout;
    c->err.clear();
    return DPMT_OK;
}

dpmt_status dpmt_set_profiling(dpmt_ctx* c, int32_t on) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (on && !c->has_device()) return fail(c, DPMT_E_STATE, "host-only context has no stream to time");
    c->prof = on != 0;
    c->ev_used = 0;
    return DPMT_OK;
}

int32_t dpmt_stage_times(dpmt_ctx* c, float* ms_out, int32_t n, int32_t* n_calls) {
    if (n_calls) *n_calls = 0;
    if (!c || !ms_out || n <= 0 || c->ev_used == 0) return 0;
    (void)hipSetDevice(c->device);
    double sum[N_STAGES + 1] = {};
    for (int k = 0; k < c->ev_used; ++k) {
        auto& ev = c->ev_sets[k];
        if (hipEventSynchronize(ev[N_STAGES]) != hipSuccess) return 0;
        float t;
        for (int i = 0; i < N_STAGES; ++i) {
            if (c->ev_whole_only[k]) {
                sum[i] = NAN;                          // one graph launch: no stage split
                continue;
            }
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) return 0;
            sum[i] += t;
        }
        if (hipEventElapsedTime(&t, ev[0], ev[N_STAGES]) != hipSuccess) return 0;
        sum[N_STAGES] += t;
    }
    const int m = std::min<int32_t>(n, N_STAGES + 1);
    for (int i = 0; i < m; ++i) ms_out[i] = (float)(sum[i] / c->ev_used);
    if (n_calls) *n_calls = c->ev_used;
    return m;
}

dpmt_status dpmt_score_pyramid(dpmt_ctx* c, dpmt_mode mode, const float* features_dev,
                               float* scores_dev, int16_t* offsets_dev, void* hip_stream) {
    dpmt_status s = score_checks(c, mode, features_dev, scores_dev);
    if (s != DPMT_OK) return s;
    hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream;
    if ((s = score_prepare(c, mode, st)) != DPMT_OK) return s;
    hipEvent_t* ev = nullptr;
    if (c->prof) {
        if (c->ev_used == (int)c->ev_sets.size()) {
            std::array<hipEvent_t, N_EVENTS> set{};
            for (auto& e : set) HIP_TRY(c, hipEventCreate(&e), "hipEventCreate");
            c->ev_sets.push_back(set);
            c->ev_whole_only.push_back(0);
        }
        c->ev_whole_only[c->ev_used] = c->launch == DPMT_LAUNCH_GRAPH;
        ev = c->ev_sets[c->ev_used++].data();
    }
    if (c->launch == DPMT_LAUNCH_GRAPH) {
        dpmt_ctx::GraphKey key;
        key.mode = mode;
        key.plan_id = c->plan_id;
        key.cfg = c->modes[mode].tile_cfg;
        key.f = features_dev;
        key.s = scores_dev;
        key.o = offsets_dev;
        if (!c->graph_exec || !(c->graph_key == key)) {
            drop_graph(c);
            if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
            HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
            hipError_t e = enqueue_batched(c, mode, features_dev, scores_dev, offsets_dev, c->cap_stream, nullptr);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                c->graph_exec = nullptr;
                return hip_fail(c, e, "graph capture");
            }
            c->graph_key = key;
        }
        if (ev) for (int k = 0; k < N_STAGES; ++k) HIP_TRY(c, hipEventRecord(ev[k], st), "hipEventRecord");
        HIP_TRY(c, hipGraphLaunch(c->graph_exec, st), "hipGraphLaunch");
        if (ev) HIP_TRY(c, hipEventRecord(ev[N_STAGES], st), "hipEventRecord");
        return DPMT_OK;
    }
    const hipError_t e =
        c->launch == DPMT_LAUNCH_PER_LEVEL ? enqueue_per_level(c, mode, features_dev, scores_dev, offsets_dev, st, ev)
        : c->launch == DPMT_LAUNCH_OVERLAP ? enqueue_overlap(c, mode, features_dev, scores_dev, offsets_dev, st, ev)
                                           : enqueue_batched(c, mode, features_dev, scores_dev, offsets_dev, st, ev);
    if (e != hipSuccess) return hip_fail(c, e, "score launch");
    return DPMT_OK;
}

dpmt_status dpmt_set_launch(dpmt_ctx* c, int32_t launch) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (launch < DPMT_LAUNCH_BATCHED || launch > DPMT_LAUNCH_OVERLAP) return fail(c, DPMT_E_INVALID, "unknown launch strategy");
    if (c->has_device() && c->graph_exec) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        drop_graph(c);
    }
    c->launch = launch;
    return DPMT_OK;
}

int32_t dpmt_tile_config_count(void) { return N_TILE_CFGS; }

const char* dpmt_tile_config_name(int32_t config) {
    return (config >= 0 && config < N_TILE_CFGS) ? TILE_CFGS[config].name : nullptr;
}

dpmt_status dpmt_set_tile_config(dpmt_ctx* c, dpmt_mode mode, int32_t config) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (mode < DPMT_DIRECT_FP32 || mode > DPMT_CP_FP32) return fail(c, DPMT_E_INVALID, "unknown mode");
    if (config < 0 || config >= N_TILE_CFGS) return fail(c, DPMT_E_INVALID, "tile configuration out of range");
    if (mode == DPMT_CP_FP32 && config != 0) return fail(c, DPMT_E_UNSUPPORTED, "the CP mode has one tile shape (configuration 0)");
    const TileCfg& tc = TILE_CFGS[config];
    int max_h = 0;
    for (const auto& sh : c->shapes) max_h = std::max(max_h, sh.h);
    if (!corr_shape_supported(tc.ty, tc.bb, tc.wy, tc.wx, max_h))
        return fail(c, DPMT_E_UNSUPPORTED, "tile configuration does not support filters of " + std::to_string(max_h) + " rows");
    c->modes[mode].tile_cfg = config;
    return DPMT_OK;
}

int32_t dpmt_get_tile_config(const dpmt_ctx* c, dpmt_mode mode) {
    if (!c || mode < DPMT_DIRECT_FP32 || mode > DPMT_CP_FP32) return -1;
    return c->modes[mode].tile_cfg;
}

dpmt_status dpmt_autotune(dpmt_ctx* c, dpmt_mode mode, const float* features_dev, float* scores_dev,
                          int16_t* offsets_dev, int32_t reps, float* ms_out, int32_t* best_out,
                          void* hip_stream) {
    dpmt_status s = score_checks(c, mode, features_dev, scores_dev);
    if (s != DPMT_OK) return s;
    if (reps < 1 || reps > 1000) return fail(c, DPMT_E_INVALID, "reps must be in [1, 1000]");
    hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream;
    ModeData& md = c->modes[mode];
    const int keep = md.tile_cfg;
    int max_h = 0;
    for (const auto& sh : c->shapes) max_h = std::max(max_h, sh.h);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(c, hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(c, hipEventCreate(&e1), "hipEventCreate");
    int best = -1;
    float best_ms = 0.f;
    hipError_t err = hipSuccess;
    for (int k = 0; k < N_TILE_CFGS && err == hipSuccess; ++k) {
        if (ms_out) ms_out[k] = -1.f;
        const TileCfg& tc = TILE_CFGS[k];
        if (!corr_shape_supported(tc.ty, tc.bb, tc.wy, tc.wx, max_h)) continue;
        if (mode == DPMT_CP_FP32 && k != 0) continue;
        md.tile_cfg = k;
        if ((s = score_prepare(c, mode, st)) != DPMT_OK) break;
        std::vector<float> t;
        for (int r = 0; r <= reps && err == hipSuccess; ++r) {        // the first run warms up
            err = hipEventRecord(e0, st);
            if (err == hipSuccess) err = enqueue_batched(c, mode, features_dev, scores_dev, offsets_dev, st, nullptr);
            if (err == hipSuccess) err = hipEventRecord(e1, st);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) t.push_back(ms);
        }
        if (err != hipSuccess) break;
        std::sort(t.begin(), t.end());
        const float med = t[t.size() / 2];
        if (ms_out) ms_out[k] = med;
        if (best < 0 || med < best_ms) {
            best = k;
            best_ms = med;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != DPMT_OK) {
        md.tile_cfg = keep;
        return s;
    }
    if (err != hipSuccess) {
        md.tile_cfg = keep;
        return hip_fail(c, err, "autotune");
    }
    md.tile_cfg = best >= 0 ? best : keep;
    if (best_out) *best_out = md.tile_cfg;
    return DPMT_OK;
}

dpmt_status dpmt_detect(dpmt_ctx* c, const float* scores_dev, float tau, dpmt_detection* dets_dev,
                        int64_t capacity, int64_t* count_dev, void* hip_stream) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (!c->planned) return fail(c, DPMT_E_STATE, "dpmt_detect before dpmt_plan");
    if (!c->has_device()) return fail(c, DPMT_E_STATE, "host-only context cannot detect");
    if (!std::isfinite(tau)) return fail(c, DPMT_E_INVALID, "tau must be finite");
    if (capacity < 0) return fail(c, DPMT_E_INVALID, "capacity must be >= 0");
    if (!count_dev || (!scores_dev && c->layout.n_score > 0) || (!dets_dev && capacity > 0))
        return fail(c, DPMT_E_INVALID, "scores_dev, count_dev and (for capacity > 0) dets_dev are required");
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream;
    static_assert(sizeof(dpmt_detection) == sizeof(Detection), "detection record layout");
    HIP_TRY(c, launch_detect(scores_dev, c->layout.n_score, tau, c->d_maps, (int)c->maps.size(),
                             c->d_det_counts, count_dev, reinterpret_cast<Detection*>(dets_dev), capacity, st),
            "detection launch");
    return DPMT_OK;
}

dpmt_status dpmt_hog_pyramid(dpmt_ctx* c, const uint8_t* image_dev, int32_t height, int32_t width,
                             int32_t n_levels, const dpmt_hog_level* levels, float* features_dev,
                             void* hip_stream) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (height < 1 || width < 1 || height > DPMT_HOG_MAX_SIDE || width > DPMT_HOG_MAX_SIDE)
        return fail(c, DPMT_E_INVALID, "image sides must be in [1, DPMT_HOG_MAX_SIDE]");
    if (n_levels < 0 || (n_levels > 0 && !levels)) return fail(c, DPMT_E_INVALID, "need levels for n_levels > 0");
    if (n_levels > 0 && (!image_dev || !features_dev))
        return fail(c, DPMT_E_INVALID, "image_dev and features_dev are required");
    std::vector<HogLevelDesc> lv((size_t)n_levels);
    std::vector<std::pair<int64_t, int64_t>> spans;
    int64_t hist_cells = 0;
    for (int l = 0; l < n_levels; ++l) {
        const dpmt_hog_level& h = levels[l];
        const std::string at = "level " + std::to_string(l) + ": ";
        if (h.cell != 4 && h.cell != 8) return fail(c, DPMT_E_INVALID, at + "cell must be 4 or 8");
        if (!std::isfinite(h.inv_scale) || !(h.inv_scale > 0.f)) return fail(c, DPMT_E_INVALID, at + "inv_scale must be finite and > 0");
        if (h.cell_offset < 0 || h.pad_rows < 0 || h.pad_cols < 0 || h.rows < 2 * (int64_t)h.pad_rows ||
            h.cols < 2 * (int64_t)h.pad_cols)
            return fail(c, DPMT_E_INVALID, at + "needs cell_offset >= 0 and rows, cols >= twice the padding");
        if (h.rows > 16384 || h.cols > 16384)
            return fail(c, DPMT_E_UNSUPPORTED, at + "sides up to 16384 cells");
        HogLevelDesc& d = lv[l];
        d.cell_offset = h.cell_offset;
        d.rows = h.rows;
        d.cols = h.cols;
        d.pad_rows = h.pad_rows;
        d.pad_cols = h.pad_cols;
        d.nr = h.rows - 2 * h.pad_rows;
        d.nc = h.cols - 2 * h.pad_cols;
        d.cell = h.cell;
        d.inv_scale = h.inv_scale;
        d.hist_off = hist_cells;
        hist_cells += (int64_t)d.nr * d.nc;
        if ((int64_t)h.rows * h.cols > 0) spans.push_back({h.cell_offset, h.cell_offset + (int64_t)h.rows * h.cols});
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k)
        if (spans[k].first < spans[k - 1].second) return fail(c, DPMT_E_INVALID, "levels overlap in the feature buffer");
    if (!c->has_device()) return fail(c, DPMT_E_STATE, "host-only context cannot extract features");
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream;
    if (n_levels == 0) return DPMT_OK;

    std::vector<int4> tiles;
    std::vector<int2> blocks;
    for (int l = 0; l < n_levels; ++l) {
        const HogLevelDesc& d = lv[l];
        const int T = HOG_TILE_PIXELS / d.cell;
        for (int ty = 0; ty < (d.nr + T - 1) / T; ++ty)
            for (int tx = 0; tx < (d.nc + T - 1) / T; ++tx) tiles.push_back(make_int4(l, ty, tx, 0));
        for (int64_t p = 0; p < (int64_t)d.rows * d.cols; p += 256) blocks.push_back(make_int2(l, (int)p));
    }
    if (tiles.size() > (size_t)INT32_MAX || blocks.size() > (size_t)INT32_MAX)
        return fail(c, DPMT_E_UNSUPPORTED, "pyramid too large for one launch");
    auto same = [](const void* a, const void* b, size_t n) { return n == 0 || std::memcmp(a, b, n) == 0; };
    const bool changed = height != c->hog_H || width != c->hog_W || lv.size() != c->hog_levels.size() ||
                         tiles.size() != c->hog_tiles.size() || blocks.size() != c->hog_blocks.size() ||
                         !same(lv.data(), c->hog_levels.data(), lv.size() * sizeof(HogLevelDesc)) ||
                         !same(tiles.data(), c->hog_tiles.data(), tiles.size() * sizeof(int4)) ||
                         !same(blocks.data(), c->hog_blocks.data(), blocks.size() * sizeof(int2));
    if (changed || hist_cells > c->hog_hist_cells) {
        // earlier calls on the stream may still read the old tables and scratch
        HIP_TRY(c, hipStreamSynchronize(st), "hipStreamSynchronize");
    }
    if (changed) {
        dfree(c->d_hog_levels); c->d_hog_levels = nullptr;
        dfree(c->d_hog_tiles); c->d_hog_tiles = nullptr;
        dfree(c->d_hog_blocks); c->d_hog_blocks = nullptr;
        c->hog_levels.clear();
        c->hog_tiles.clear();
        c->hog_blocks.clear();
        c->hog_H = c->hog_W = -1;
        auto put = [&](void** dst, const void* src, size_t bytes, const char* what) -> dpmt_status {
            if (bytes == 0) return DPMT_OK;
            hipError_t e = hipMalloc(dst, bytes);
            if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
            return e == hipSuccess ? DPMT_OK : hip_fail(c, e, what);
        };
        dpmt_status s;
        if ((s = put((void**)&c->d_hog_levels, lv.data(), lv.size() * sizeof(HogLevelDesc), "upload HOG levels")) != DPMT_OK) return s;
        if ((s = put((void**)&c->d_hog_tiles, tiles.data(), tiles.size() * sizeof(int4), "upload HOG tiles")) != DPMT_OK) return s;
        if ((s = put((void**)&c->d_hog_blocks, blocks.data(), blocks.size() * sizeof(int2), "upload HOG blocks")) != DPMT_OK) return s;
        c->hog_levels = lv;
        c->hog_tiles = tiles;
        c->hog_blocks = blocks;
        c->hog_H = height;
        c->hog_W = width;
    }
    if (hist_cells > c->hog_hist_cells) {
        dfree(c->d_hog_hist); c->d_hog_hist = nullptr; c->hog_hist_cells = 0;
        HIP_TRY(c, hipMalloc((void**)&c->d_hog_hist, (size_t)hist_cells * 19 * sizeof(float)), "allocate HOG scratch");
        c->hog_hist_cells = hist_cells;
    }
    HogTable tab;
    for (int o = 0; o < 9; ++o) {
        tab.u[o] = (float)std::cos(o * M_PI / 9.0);
        tab.v[o] = (float)std::sin(o * M_PI / 9.0);
    }
    float* hist = c->d_hog_hist;
    float* energy = hist ? hist + c->hog_hist_cells * 18 : nullptr;
    HIP_TRY(c, launch_hog(image_dev, height, width, c->d_hog_levels, c->d_hog_tiles, (int)tiles.size(),
                          c->d_hog_blocks, (int)blocks.size(), tab, hist, energy, features_dev, st),
            "HOG launch");
    return DPMT_OK;
}

dpmt_status dpmt_level_responses(dpmt_ctx* c, dpmt_mode mode, const float* features_dev,
                                 int32_t image, int32_t level, float* out_dev, int64_t capacity,
                                 int64_t* n_written, void* hip_stream) {
    if (!c) return fail(nullptr, DPMT_E_INVALID, "ctx is NULL");
    if (mode < DPMT_DIRECT_FP32 || mode > DPMT_CP_FP32) return fail(c, DPMT_E_INVALID, "unknown mode");
    if (!c->loaded) return fail(c, DPMT_E_STATE, "dpmt_level_responses before dpmt_load_filters");
    if (is_tensor(mode) && !c->decomposed) return fail(c, DPMT_E_STATE, "tensor mode needs dpmt_decompose first");
    if (mode == DPMT_CP_FP32 && !c->cp_ready) return fail(c, DPMT_E_STATE, "CP mode needs dpmt_decompose_cp or dpmt_load_cp first");
    if (!c->planned) return fail(c, DPMT_E_STATE, "dpmt_level_responses before dpmt_plan");
    if (!c->has_device()) return fail(c, DPMT_E_STATE, "host-only context cannot compute");
    if (image < 0 || image >= (int)c->pyr.size()) return fail(c, DPMT_E_INVALID, "image out of range");
    if (level < 0 || level >= (int)c->pyr[image].size()) return fail(c, DPMT_E_INVALID, "level out of range");
    const LevelInfo lv = c->pyr[image][level];
    std::vector<int64_t> map_off(c->shapes.size(), -1);
    int64_t total = 0;
    for (size_t k = 0; k < c->shapes.size(); ++k) {
        const int Ho = lv.rows - c->shapes[k].h + 1, Wo = lv.cols - c->shapes[k].w + 1;
        if (Ho <= 0 || Wo <= 0) continue;
        map_off[k] = total;
        total += (int64_t)Ho * Wo;
    }
    if (n_written) *n_written = total;
    if (!out_dev && capacity == 0) return DPMT_OK;            // size query
    if (!features_dev || !out_dev) return fail(c, DPMT_E_INVALID, "features_dev and out_dev are required");
    if (capacity < total) return fail(c, DPMT_E_INVALID, "out_dev capacity " + std::to_string(capacity) + " < " + std::to_string(total));
    HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
    dpmt_status s = prepare_mode(c, mode);
    if (s != DPMT_OK) return s;
    ModeData& md = c->modes[mode];
    hipStream_t st = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream;
    const bool tensor = is_tensor(mode);
    // per-group planes in a temporary buffer, then copied to per-filter maps
    std::vector<CorrTile> tiles;
    std::vector<CpTile> cp_tiles;
    struct GB { int g; int64_t off; int Ho, Wo, ld; };
    std::vector<GB> gblocks;
    int64_t blk_total = 0;
    int max_h = 0, max_S = 0;
    for (size_t g = 0; g < c->groups.size(); ++g) {
        if (c->groups[g].role != ROLE_ALL) continue;
        const HostGroup& hg = c->groups[g];
        const int Ho = lv.rows - hg.h + 1, Wo = lv.cols - hg.w + 1;
        if (Ho <= 0 || Wo <= 0) continue;
        if (mode == DPMT_CP_FP32) {
            add_cp_tiles(cp_tiles, hg, md.cp_chunk0[g], lv.cell_offset, blk_total, -1, lv.rows, lv.cols);
        } else {
            const GroupDesc& gd = md.groups[g];
            add_tiles(tiles, gd, (int)g, 0, blk_total, -1, lv.rows, lv.cols, 16, 32, 2, 1);
            max_S = std::max(max_S, gd.S);
        }
        gblocks.push_back({(int)g, blk_total, Ho, Wo, pitch_of(Wo)});
        blk_total += (int64_t)Ho * pitch_of(Wo) * (int64_t)hg.filters.size();
        max_h = std::max(max_h, hg.h);
    }
    if (tiles.empty() && cp_tiles.empty()) return DPMT_OK;
    const int64_t cells = (int64_t)lv.rows * lv.cols;
    void* dZ = nullptr;
    float* dblk = nullptr;
    CorrTile* dtiles = nullptr;
    CpTile* dcp = nullptr;
    int64_t* doff = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        dfree(dZ); dfree(dblk); dfree(dtiles); dfree(dcp); dfree(doff);
    };
    hipError_t e = hipSuccess;
    const void* Zsrc = features_dev + lv.cell_offset * 32;
    if (tensor) {
        e = hipMalloc(&dZ, (size_t)cells * md.pk.RP * md.pk.esz);
        if (e == hipSuccess) {
            if (mode == DPMT_TENSOR_FP8) e = fp8_operands(md, features_dev + lv.cell_offset * 32, cells, dZ, nullptr, 0, st);
            else e = launch_project(md.pk.esz == 2, features_dev + lv.cell_offset * 32, cells, md.dU, md.pk.RP, dZ,
                                    nullptr, 0, st);
        }
        Zsrc = dZ;
    }
    if (e == hipSuccess) e = hipMalloc((void**)&dblk, (size_t)blk_total * 4);
    if (mode == DPMT_CP_FP32) {
        size_t lds = 0;
        for (const CpTile& t : cp_tiles) lds = std::max(lds, cp_lds_bytes(t.HX, t.HY));
        if (e == hipSuccess) e = upload(&dcp, cp_tiles);
        if (e == hipSuccess) e = launch_cp_corr(dcp, (int)cp_tiles.size(), md.dCpChunks, features_dev, md.dCpFac, dblk, nullptr, 0, nullptr, lds, st);
    } else {
        if (e == hipSuccess) e = upload(&dtiles, tiles);
        CorrLaunch cl{md.kind, md.pk, 4, 2, 4, 0, 1, 0};
        if (e == hipSuccess) e = launch_corr(cl, dtiles, (int)tiles.size(), md.dGroups, Zsrc, md.dG, md.dTk, dblk, nullptr, 0, max_h, max_S, st);
    }
    for (const auto& gb : gblocks) {
        if (e != hipSuccess) break;
        const HostGroup& hg = c->groups[gb.g];
        std::vector<int64_t> dst;
        for (int k : hg.filters) dst.push_back(map_off[k]);
        dfree(doff);
        doff = nullptr;
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = upload(&doff, dst);
        if (e == hipSuccess) e = launch_planes_to_maps(dblk + gb.off, (int)hg.filters.size(), gb.Ho, gb.Wo, gb.ld, doff, out_dev, st);
    }
    cleanup();
    if (e != hipSuccess) return hip_fail(c, e, "level responses");
    return DPMT_OK;
}

}  // extern "C"

namespace {
// Arguments of the single-map transform (both entry points).
dpmt_status check_dt_args(const float* resp_dev, int32_t rows, int32_t cols, int32_t ld,
                          const float* deform_host, const float* d_dev, const int32_t* arg_y_dev,
                          const int32_t* arg_x_dev) {
    if (!resp_dev || !deform_host || !d_dev) return fail(nullptr, DPMT_E_INVALID, "resp_dev, deform_host and d_dev are required");
    if (rows < 1 || cols < 1 || ld < cols) return fail(nullptr, DPMT_E_INVALID, "need rows >= 1, cols >= 1, ld >= cols");
    if ((arg_y_dev == nullptr) != (arg_x_dev == nullptr)) return fail(nullptr, DPMT_E_INVALID, "arg_y_dev and arg_x_dev must both be given or both NULL");
    for (int t = 0; t < 4; ++t)
        if (!std::isfinite(deform_host[t])) return fail(nullptr, DPMT_E_INVALID, "non-finite deformation coefficient");
    if (!(deform_host[1] > 0.f) || !(deform_host[3] > 0.f)) return fail(nullptr, DPMT_E_INVALID, "quadratic deformation coefficients must be > 0");
    if ((int64_t)rows * cols > (int64_t)1 << 30) return fail(nullptr, DPMT_E_UNSUPPORTED, "map larger than 2^30 cells");
    return DPMT_OK;
}
}  // namespace

extern "C" {

dpmt_status dpmt_distance_transform(const float* resp_dev, int32_t rows, int32_t cols, int32_t ld,
                                    const float* deform_host, float* d_dev, int32_t* arg_y_dev,
                                    int32_t* arg_x_dev, void* hip_stream) {
    const dpmt_status chk = check_dt_args(resp_dev, rows, cols, ld, deform_host, d_dev, arg_y_dev, arg_x_dev);
    if (chk != DPMT_OK) return chk;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t n = (int64_t)rows * cols;
    float* lmax = nullptr;
    float* r1v = nullptr;
    int32_t* r1a = nullptr;
    hipError_t e = hipMallocAsync((void**)&lmax, (size_t)std::max(rows, cols) * 4, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&r1v, (size_t)n * 4, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&r1a, (size_t)n * 4, st);
    if (e == hipSuccess) e = launch_dt_single(resp_dev, rows, cols, ld, deform_host, lmax, r1v, r1a, d_dev, arg_y_dev, arg_x_dev, st);
    if (lmax) (void)hipFreeAsync(lmax, st);
    if (r1v) (void)hipFreeAsync(r1v, st);
    if (r1a) (void)hipFreeAsync(r1a, st);
    if (e != hipSuccess) return hip_fail(nullptr, e, "distance transform");
    return DPMT_OK;
}

dpmt_status dpmt_distance_transform_method(const float* resp_dev, int32_t rows, int32_t cols, int32_t ld,
                                           const float* deform_host, float* d_dev, int32_t* arg_y_dev,
                                           int32_t* arg_x_dev, int32_t method, void* hip_stream) {
    if (method == DPMT_DT_WINDOW)
        return dpmt_distance_transform(resp_dev, rows, cols, ld, deform_host, d_dev, arg_y_dev, arg_x_dev,
                                       hip_stream);
    if (method != DPMT_DT_ENVELOPE) return fail(nullptr, DPMT_E_INVALID, "unknown distance transform method");
    const dpmt_status chk = check_dt_args(resp_dev, rows, cols, ld, deform_host, d_dev, arg_y_dev, arg_x_dev);
    if (chk != DPMT_OK) return chk;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t n = (int64_t)rows * cols;
    float* r1v = nullptr;
    int32_t* r1a = nullptr;
    int32_t* hx = nullptr;
    double* hz = nullptr;
    int32_t* ayw = nullptr;
    hipError_t e = hipMallocAsync((void**)&r1v, (size_t)n * 4, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&r1a, (size_t)n * 4, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&hx, (size_t)n * 4, st);
    if (e == hipSuccess) e = hipMallocAsync((void**)&hz, (size_t)n * 8, st);
    if (e == hipSuccess && !arg_y_dev) e = hipMallocAsync((void**)&ayw, (size_t)n * 4, st);
    if (e == hipSuccess)
        e = launch_dt_envelope(resp_dev, rows, cols, ld, deform_host, r1v, r1a, hx, hz, d_dev,
                               arg_y_dev ? arg_y_dev : ayw, arg_x_dev, st);
    for (void* p : {(void*)r1v, (void*)r1a, (void*)hx, (void*)hz, (void*)ayw})
        if (p) (void)hipFreeAsync(p, st);
    if (e != hipSuccess) return hip_fail(nullptr, e, "distance transform (lower envelopes)");
    return DPMT_OK;
}

dpmt_status dpmt_distance_transform_noalloc(const float* resp_dev, int32_t rows, int32_t cols,
                                            int32_t ld, const float* deform_host, float* d_dev,
                                            int32_t* arg_y_dev, int32_t* arg_x_dev, void* hip_stream) {
    const dpmt_status chk = check_dt_args(resp_dev, rows, cols, ld, deform_host, d_dev, arg_y_dev, arg_x_dev);
    if (chk != DPMT_OK) return chk;
    if (rows > DT_NOALLOC_MAX_SIDE || cols > DT_NOALLOC_MAX_SIDE)
        return fail(nullptr, DPMT_E_UNSUPPORTED, "allocation-free transform: rows and cols must be <= 16384");
    if ((int64_t)rows * cols > DT_NOALLOC_MAX_CELLS)
        return fail(nullptr, DPMT_E_UNSUPPORTED, "allocation-free transform: map larger than 2^21 cells");
    const hipError_t e = launch_dt_single_noalloc(resp_dev, rows, cols, ld, deform_host, d_dev, arg_y_dev,
                                                  arg_x_dev, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(nullptr, e, "allocation-free distance transform");
    return DPMT_OK;
}

}  // extern "C"
