/*
 * dpmt.h -- C ABI of libdpmt, DPM score estimation on AMD MI355X (gfx950).
 *
 * The library computes, for every root position of every level of a HOG
 * feature pyramid and every mixture component, the star-model score
 *     s(p0) = f0 . phi(p0) + sum_i ( f_i . phi(p_i) - d_i . psi(p_i, p0) )
 * with every part placed at its best position (Section 2, the score formula
 * and the placement argmax over all part positions).  Filter responses are
 * computed either directly or in the tensor form of Section 4: the filter
 * bank is decomposed once into a shared feature-mode basis U_R (the leading
 * R eigenvectors of the Gram matrix of the bank's mode-3 unfolding, the
 * Frobenius-optimal truncation of that mode), features are projected onto it
 * once per level, and rank-R correlations replace the 32-channel ones.
 *
 * Conventions used throughout:
 *   - A feature level is rows x cols cells of 32 float32 channels, channel
 *     innermost (HWC).  A filter is h x w x 32 float32, HWC.
 *   - A response is a correlation (not a convolution) over valid placements:
 *     resp(y, x) = sum_{n<h, m<w, l<32} f[n][m][l] * X[y+n][x+m][l],
 *     0 <= y <= rows-h, 0 <= x <= cols-w.
 *   - Deformation coefficients d = (d_x, d_xx, d_y, d_yy); the cost of a part
 *     at (y', x') for anchor (ya, xa) is
 *     d_x*(x'-xa) + d_xx*(x'-xa)^2 + d_y*(y'-ya) + d_yy*(y'-ya)^2.
 *   - Parts of a root at pyramid level l live on level l - octave, at twice
 *     the resolution: the anchor of part i for root position (y0, x0) is
 *     (2*y0 + v_y, 2*x0 + v_x).  An anchor outside the part response map
 *     gives score -inf.  Ties in the placement argmax go to the smallest
 *     (y', x') in lexicographic order.
 *
 * Memory: every pointer argument is owned by the caller and never freed by
 * the library.  "_host" pointers are host memory, read during the call and
 * copied where kept.  "_dev" pointers are device memory on the context's
 * GPU.  Calls that take a hip_stream (a hipStream_t, NULL = the context's
 * stream) enqueue work asynchronously on it; validation happens before
 * anything is enqueued, and a failed validation leaves outputs untouched.
 * A context is not thread-safe; different contexts are independent.
 */
#ifndef DPMT_H
#define DPMT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dpmt_ctx dpmt_ctx;

typedef enum {
    DPMT_OK = 0,
    DPMT_E_INVALID = -1,      /* bad argument: NULL pointer, bad size, bad coefficient  */
    DPMT_E_STATE = -2,        /* call out of order (e.g. score before plan)              */
    DPMT_E_RANK = -3,         /* rank outside [1, 32]                                    */
    DPMT_E_NOMEM = -4,        /* device or host allocation failed                        */
    DPMT_E_DEVICE = -5,       /* a HIP call failed; dpmt_last_error names it             */
    DPMT_E_UNSUPPORTED = -6   /* valid request this build does not handle                */
} dpmt_status;

typedef enum {
    DPMT_DIRECT_FP32 = 0,     /* 32-channel correlation, FP32 MFMA, FP32 accumulation    */
    DPMT_TENSOR_FP32 = 1,     /* rank-R tensor form, FP32 projection and MFMA            */
    DPMT_TENSOR_BF16 = 2,     /* rank-R tensor form, BF16 operands, FP32 accumulation    */
    DPMT_TENSOR_FP8 = 3,      /* rank-R tensor form, FP8 e4m3 operands with per-channel
                                 scales, FP32 accumulation                               */
    DPMT_CP_FP32 = 4          /* per-filter CP form (Section 4): each filter a sum of R_k
                                 outer products a (x) b (x) c; channel contraction on FP32
                                 MFMA, then 1-D correlations along x and y, FP32        */
} dpmt_mode;

/* How dpmt_score_pyramid issues its work (dpmt_set_launch).  Every strategy
 * runs the same kernels on the same tiles and produces the same bits. */
typedef enum {
    DPMT_LAUNCH_BATCHED = 0,  /* one launch per stage over every level of every image:
                                 projection (which also resets the value ranges; a reset
                                 kernel of its own in the direct, FP8 and CP modes),
                                 correlation, placement                                  */
    DPMT_LAUNCH_PER_LEVEL = 1,/* projection and correlation launched per (image, level),
                                 placement per (image, root level): the reference for
                                 what batching saves                                     */
    DPMT_LAUNCH_GRAPH = 2,    /* the batched launches captured once into a HIP graph and
                                 replayed; re-captured when the mode, plan, tile
                                 configuration or a device pointer changes               */
    DPMT_LAUNCH_OVERLAP = 3   /* (image, root level) dependency groups cut into chunks:
                                 correlation chunks on hip_stream, each chunk's placement
                                 on a second stream of the context once that chunk is
                                 done, joined back into hip_stream before the call ends  */
} dpmt_launch;

typedef struct { int32_t h, w; } dpmt_shape;          /* filter rows, cols; 32 channels */

/* One mixture component (Section 2: a root filter f0, n > 0 part filters f_i
 * and deformation coefficients d_i). */
typedef struct {
    int32_t        root;       /* filter index of the root filter                       */
    int32_t        n_parts;    /* >= 1                                                   */
    const int32_t* parts;      /* [n_parts] filter indices (host)                        */
    const int32_t* anchors;    /* [n_parts][2] (v_y, v_x), part-level cells (host);
                                  0 <= v_y <= 2*h0 - h_i, 0 <= v_x <= 2*w0 - w_i         */
    const float*   deform;     /* [n_parts][4] (d_x, d_xx, d_y, d_yy) (host); d_xx > 0,
                                  d_yy > 0, all finite                                   */
} dpmt_component;

typedef struct {
    int64_t cell_offset;       /* first cell of the level in the packed feature buffer  */
    int32_t rows, cols;        /* >= 1                                                   */
} dpmt_level;

typedef struct {
    int32_t           n_levels;
    const dpmt_level* levels;  /* [n_levels] (host)                                      */
    int32_t           octave;  /* levels per octave: parts of root level l use l-octave  */
} dpmt_pyramid;

/* Output layout, computed by dpmt_plan and owned by the context (valid until
 * the next dpmt_plan or dpmt_destroy).  One score map per (image, root level
 * l >= octave, component), in that nesting order; map k has map_rows[k] x
 * map_cols[k] = (rows_l - h0 + 1) x (cols_l - w0 + 1) float32 scores, row
 * major, at scores_dev + map_score_off[k] (0 x 0 when the root filter does not
 * fit), and n_parts int16 (dy, dx) placement offsets per position at
 * offsets_dev + map_offs_off[k], laid out [part][row][col][2]. */
typedef struct {
    int64_t        n_score;        /* float32 elements scores_dev must hold            */
    int64_t        n_offsets;      /* int16 elements offsets_dev must hold             */
    int32_t        n_maps;
    const int32_t* map_image;      /* [n_maps]                                         */
    const int32_t* map_level;      /* [n_maps] root level                              */
    const int32_t* map_comp;       /* [n_maps] component index                         */
    const int32_t* map_rows;       /* [n_maps]                                         */
    const int32_t* map_cols;       /* [n_maps]                                         */
    const int64_t* map_score_off;  /* [n_maps] element offsets into scores_dev         */
    const int64_t* map_offs_off;   /* [n_maps] element offsets into offsets_dev        */
    int64_t        n_cells;        /* cells (x32 floats) the feature buffer must hold  */
    int64_t        n_resp;         /* filter-response cells per dpmt_score_pyramid     */
    int64_t        n_resp_root;    /*   of which root filters on levels >= octave      */
    int64_t        n_resp_part;    /*   of which part filters one octave below         */
    int64_t        workspace_bytes;/* device workspace the context holds for the plan  */
} dpmt_layout;

/* Create a context on HIP device `device` (>= 0), or a host-only context
 * (device = -1) that can load, decompose and plan but not score.  The stream
 * (a hipStream_t, may be NULL) becomes the default for calls that get NULL. */
dpmt_status dpmt_create(dpmt_ctx** out, int32_t device, void* hip_stream);
void        dpmt_destroy(dpmt_ctx* ctx);

/* Load the filter bank and the mixture components (Section 2 model).
 * weights_host: all filters concatenated, filter k is shapes[k].h x
 * shapes[k].w x 32 float32 HWC; copied.  Every weight must be finite, every
 * shape >= 1 x 1, every component index in range, d_xx > 0 and d_yy > 0,
 * anchors inside [0, 2*h0 - h_i] x [0, 2*w0 - w_i].  Replaces any previous
 * bank and drops any decomposition and plan. */
dpmt_status dpmt_load_filters(dpmt_ctx* ctx, int32_t n_filters, const dpmt_shape* shapes,
                              const float* weights_host, int32_t n_components,
                              const dpmt_component* comps);

/* Decompose the loaded bank for the tensor modes (Section 4 criterion applied
 * to the feature mode): FP64 Gram matrix C = M^T M of the mode-3 unfolding M
 * (one row per filter cell), cyclic Jacobi eigen-solve, U_R = leading `rank`
 * eigenvectors (largest-magnitude entry of each column positive), factors
 * G_k = f_k x_3 U_R^T.  sigma_out (host, may be NULL) receives the 32 singular
 * values sqrt(lambda) in descending order; basis_out (host, may be NULL)
 * receives U_R as 32 x rank row-major float64.  Uploads the quantised factors
 * when the context has a device. */
dpmt_status dpmt_decompose(dpmt_ctx* ctx, int32_t rank, double* sigma_out, double* basis_out);

/* Per-filter CP form (Section 4).  Filter k (h x w x 32) is approximated by
 *     sum_{r < R_k} a_r (x) b_r (x) c_r,   a_r in R^h, b_r in R^w, c_r in R^32,
 * and its response by the decomposed correlation: per term, the channel
 * contraction X . c_r, a 1-D correlation along x with b_r and one along y
 * with a_r, summed over r.  Factor layout (host float32, used by
 * dpmt_load_cp and dpmt_get_cp): filter after filter in bank order, each as
 * A (h x R_k), then B (w x R_k), then C (32 x R_k), all row major (A[n][r],
 * B[m][r], C[l][r]); sum_k R_k (h_k + w_k + 32) floats in all.
 *
 * dpmt_decompose_cp fits the factors in FP64 on the host by alternating least
 * squares: starting from the leading left singular vectors of the three
 * unfoldings, each cycle solves A, then B, then C as linear least-squares
 * problems (minimum-norm solutions) with the other two fixed; it stops after
 * max_iters (>= 1) cycles, once ||f - CP(f)||_F <= tol * ||f||_F (tol >= 0),
 * or when a cycle no longer lowers that error.  ranks: [n_filters] values in
 * [1, 32] (DPMT_E_RANK otherwise).  rel_err_out (host, may be NULL) receives
 * ||f_k - CP(f_k)||_F / ||f_k||_F per filter.  dpmt_load_cp takes factors
 * computed elsewhere instead (every value finite).  Either call replaces the
 * previous CP factors; dpmt_load_filters drops them. */
dpmt_status dpmt_decompose_cp(dpmt_ctx* ctx, const int32_t* ranks, int32_t max_iters, double tol,
                              double* rel_err_out);
dpmt_status dpmt_load_cp(dpmt_ctx* ctx, const int32_t* ranks, const float* factors_host);
/* Per-filter rank selection (Section 4 criterion): for every filter the
 * smallest r in [1, r_max] (r_max <= 32) with
 *     ||f - CP(f, r)||_F < e * (r (h + w + 32) / (h w 32))^2,
 * found by binary search over r (each probe an ALS fit as in
 * dpmt_decompose_cp with tol 1e-13 and max_iters cycles); r_max when no
 * rank meets it.  The fits of the chosen ranks become the CP factors, as
 * after dpmt_decompose_cp.  ranks_out ([n_filters]) and rel_err_out
 * ([n_filters], relative Frobenius errors) may be NULL. */
dpmt_status dpmt_select_ranks(dpmt_ctx* ctx, double e, int32_t r_max, int32_t max_iters,
                              int32_t* ranks_out, double* rel_err_out);
/* Current CP factors: *n_floats receives their count; ranks_out ([n_filters])
 * and factors_out (that many floats) may be NULL.  DPMT_E_STATE without CP
 * factors. */
dpmt_status dpmt_get_cp(const dpmt_ctx* ctx, int32_t* ranks_out, float* factors_out,
                        int64_t* n_floats);

/* Convolution shortening (Section 4 thresholds, Algorithm 1's early exit),
 * for DPMT_CP_FP32.  Filter k has thresholds t_1 .. t_{R_k}; a root position
 * is rejected (score -inf, every offset 0) when, for its root filter at the
 * position or for a part filter at its anchor 2 p0 + v_i (when inside the
 * part map), the sum of the first r terms' responses is below t_r for some r.
 * Other positions keep the scores and offsets the CP mode computes without
 * thresholds.  Layout: filter after filter in bank order, R_k floats each
 * (sum_k R_k in all); -inf disables a test, NaN is rejected.
 * dpmt_set_thresholds copies them (NULL clears them); new CP factors clear
 * them too.  Rejection is decided in FP32 partial sums, in term order. */
dpmt_status dpmt_set_thresholds(dpmt_ctx* ctx, const float* thresholds_host);

/* One hypothesis: root position (y, x) of component `comp` on root level
 * `level` of image `image` of the current plan. */
typedef struct {
    int32_t image, level, comp, y, x;
} dpmt_hypothesis;

/* Thresholds from positives (Section 4): t_r of filter k = the smallest
 * partial sum p_r of k over the positives whose component uses it (the root
 * at the position, each part at its anchor when inside the part map),
 * computed in FP64 on the host from features_host (the packed FP32 cells of
 * the plan), minus margin (>= 0, so that FP32 partial sums on the GPU do not
 * reject a positive); -inf for filters no positive covers.  Sets them as
 * dpmt_set_thresholds does; thresholds_out (host, sum_k R_k floats, may be
 * NULL) receives them.  Needs CP factors and a plan. */
dpmt_status dpmt_fit_thresholds(dpmt_ctx* ctx, const float* features_host, int32_t n_pos,
                                const dpmt_hypothesis* positives, float margin, float* thresholds_out);

/* Plan a batch of n_images pyramids (host descriptors, copied): output layout,
 * work lists and device workspace.  *out points at the context-owned layout.
 * Limits (DPMT_E_UNSUPPORTED beyond them): level sides up to 16384 cells,
 * part response maps up to 1976 columns, and score maps whose placement
 * working set (map height and part map height) fits one workgroup's 160 KB
 * of LDS, which holds part maps up to about 550 rows. */
dpmt_status dpmt_plan(dpmt_ctx* ctx, int32_t n_images, const dpmt_pyramid* pyrs,
                      const dpmt_layout** out);

/* Score the planned batch.  features_dev: packed float32 HWC cells (at least
 * layout->n_cells x 32).  scores_dev: layout->n_score float32.  offsets_dev:
 * layout->n_offsets int16 (may be NULL to skip placements).  Tensor modes need
 * dpmt_decompose first, DPMT_CP_FP32 dpmt_decompose_cp or dpmt_load_cp
 * (else DPMT_E_STATE). */
dpmt_status dpmt_score_pyramid(dpmt_ctx* ctx, dpmt_mode mode, const float* features_dev,
                               float* scores_dev, int16_t* offsets_dev, void* hip_stream);

/* One detection: root position (y, x) of score map `map` (a layout index)
 * and its score; the parts' placements are the map's offsets at (y, x). */
typedef struct {
    int32_t map;
    int32_t y, x;
    float   score;
} dpmt_detection;

/* Detection set of Algorithm 1: every root position of every planned score
 * map whose score is >= tau (finite), in (map, row, column) order, from the
 * scores of a dpmt_score_pyramid call enqueued before it on the same stream.
 * dets_dev receives the first min(count, capacity) records; count_dev (device,
 * one int64) receives the full count.  Asynchronous on hip_stream; uses the
 * context's scratch, so calls on one context must not overlap. */
dpmt_status dpmt_detect(dpmt_ctx* ctx, const float* scores_dev, float tau, dpmt_detection* dets_dev,
                        int64_t capacity, int64_t* count_dev, void* hip_stream);

/* One level of a HOG feature pyramid: rows x cols cells (padding included)
 * starting at cell cell_offset of a packed float32 HWC buffer of 32 channels.
 * The rows - 2 pad_rows x cols - 2 pad_cols interior cells cover the image
 * resized by 1 / inv_scale, cell x cell resized pixels each; the padding band
 * of pad_rows rows and pad_cols columns on every side gets channel 31 = 1 and
 * the other channels 0. */
typedef struct {
    int64_t cell_offset;
    int32_t rows, cols;
    int32_t pad_rows, pad_cols;
    int32_t cell;        /* 4 or 8 */
    float   inv_scale;   /* source pixels per resized pixel, finite, > 0 */
} dpmt_hog_level;

/* HOG features of an image, level by level: the feature map phi the scores
 * are computed on (Section 2), 32 values per cell (Section 5, L = 32), in
 * the 32-value variant of Felzenszwalb et al. (PAMI 2010, Section 6).  Each
 * level samples the image bilinearly at its scale; per pixel the colour
 * channel with the largest centred gradient votes for the nearest of 18
 * directions, its magnitude spread bilinearly over the 4 nearest cells; the
 * cell histograms are normalised by the 4 2x2-cell blocks around each cell,
 * truncated at 0.2 and projected to 18 contrast-sensitive, 9 insensitive and
 * 4 texture channels (channel 31 zero inside the image).
 * image_dev: height x width x 3 uint8 (RGB, row-major, no pitch).
 * levels_host: n_levels descriptors (copied); their cell ranges must not
 * overlap (DPMT_E_INVALID).  features_dev receives every level's cells; cells
 * outside the levels are not written.  Sides: image up to DPMT_HOG_MAX_SIDE
 * pixels, levels up to 16384 cells (DPMT_E_UNSUPPORTED beyond).  Needs a
 * context with a device (nothing loaded or planned); the context keeps the
 * level tables and a histogram scratch of 76 bytes per interior cell, which
 * grows when a call needs more (such a call first waits for the stream).
 * Asynchronous on hip_stream; calls on one context must not overlap. */
#define DPMT_HOG_MAX_SIDE 65536
dpmt_status dpmt_hog_pyramid(dpmt_ctx* ctx, const uint8_t* image_dev, int32_t height, int32_t width,
                             int32_t n_levels, const dpmt_hog_level* levels_host, float* features_dev,
                             void* hip_stream);

/* Filter responses of every filter of the bank on one planned level (for
 * checking the correlation stage on its own).  out_dev receives, for filter
 * k = 0 .. n_filters-1 in order, its (rows - h_k + 1) x (cols - w_k + 1)
 * row-major float32 map (nothing for a filter that does not fit); capacity is
 * out_dev's size in elements (DPMT_E_INVALID if too small).  n_written (host,
 * may be NULL) receives the element count; out_dev = NULL with capacity = 0
 * only reports that count. */
dpmt_status dpmt_level_responses(dpmt_ctx* ctx, dpmt_mode mode, const float* features_dev,
                                 int32_t image, int32_t level, float* out_dev,
                                 int64_t capacity, int64_t* n_written, void* hip_stream);

/* Generalised distance transform of one map (Section 2 placement argmax for
 * every target cell): d_dev[y][x] = max over all (y', x') of
 * resp[y'][x'] - cost(y'-y, x'-x), with arg_y_dev / arg_x_dev the maximiser
 * (int32, may both be NULL).  resp_dev is rows x cols float32 with row pitch
 * ld >= cols elements; outputs are rows x cols, pitch cols.  deform_host is
 * (d_x, d_xx, d_y, d_yy) with d_xx > 0, d_yy > 0.  FP32 arithmetic. */
dpmt_status dpmt_distance_transform(const float* resp_dev, int32_t rows, int32_t cols, int32_t ld,
                                    const float* deform_host, float* d_dev, int32_t* arg_y_dev,
                                    int32_t* arg_x_dev, void* hip_stream);

/* dpmt_distance_transform with a choice of method: DPMT_DT_WINDOW is
 * dpmt_distance_transform itself (exact scans of the window that the line's
 * value range allows, work growing with sqrt(range / d_xx) per target);
 * DPMT_DT_ENVELOPE finds the same maximum along each line from the upper
 * envelope of the candidates' cost parabolas (Section 2 placement argmax,
 * computed as in Felzenszwalb and Huttenlocher's distance transform of
 * sampled functions), in time linear in the line length whatever the
 * deformation, one GPU thread per line.  The envelope is built in FP64 and
 * the maximiser is decided in FP32 among the envelope's candidates with the
 * window scan's formula and tie rule, so both methods agree wherever the
 * FP32 values of the top two candidates differ.  Inputs finite or -inf (an
 * all -inf line gives -inf).  Other arguments as dpmt_distance_transform;
 * an unknown method is DPMT_E_INVALID. */
#define DPMT_DT_WINDOW 0
#define DPMT_DT_ENVELOPE 1
dpmt_status dpmt_distance_transform_method(const float* resp_dev, int32_t rows, int32_t cols, int32_t ld,
                                           const float* deform_host, float* d_dev, int32_t* arg_y_dev,
                                           int32_t* arg_x_dev, int32_t method, void* hip_stream);

/* dpmt_distance_transform for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, kernels and results, but the scratch the transform needs
 * (line maxima and the row pass's values and argmax, 16 MiB + 64 KiB) lives
 * in a static device array of the library that each GPU holds from its first
 * use until the process ends; the call allocates nothing.  Runs on the
 * current HIP device (hip_stream must belong to it); the first call on a
 * device looks up that device's copy of the array.  Limits:
 * rows <= DPMT_DT_NOALLOC_MAX_SIDE, cols <= DPMT_DT_NOALLOC_MAX_SIDE and
 * rows * cols <= DPMT_DT_NOALLOC_MAX_CELLS, else DPMT_E_UNSUPPORTED before
 * anything is enqueued.  Every call on a GPU uses that GPU's one array, so
 * calls that overlap on one GPU (other streams, other threads) race: order
 * them on one stream or synchronise between them. */
#define DPMT_DT_NOALLOC_MAX_SIDE 16384
#define DPMT_DT_NOALLOC_MAX_CELLS 2097152
dpmt_status dpmt_distance_transform_noalloc(const float* resp_dev, int32_t rows, int32_t cols,
                                            int32_t ld, const float* deform_host, float* d_dev,
                                            int32_t* arg_y_dev, int32_t* arg_x_dev,
                                            void* hip_stream);

/* Per-stage GPU timing from HIP events recorded on the launch stream around
 * each stage of dpmt_score_pyramid.  dpmt_set_profiling(ctx, 1) starts
 * recording (and clears what was gathered); every later score call adds one
 * set of events.  dpmt_stage_times waits for the recorded events and writes
 * the mean duration per call, in milliseconds, of each stage: 0 projection
 * (with the reset of the per-plane value ranges), 1 correlation (all filters
 * of all levels), 2 placement (distance transform at the anchors and score
 * assembly), 3 whole call.  Returns the number of stages written (at most n)
 * and stores the number of calls averaged in *n_calls (may be NULL). */
dpmt_status dpmt_set_profiling(dpmt_ctx* ctx, int32_t on);
int32_t     dpmt_stage_times(dpmt_ctx* ctx, float* ms_out, int32_t n, int32_t* n_calls);

/* Launch strategy of later dpmt_score_pyramid calls (a dpmt_launch value;
 * DPMT_E_INVALID otherwise).  In graph mode the per-stage times of
 * dpmt_stage_times are NaN (one launch) and only the whole-call time is kept. */
dpmt_status dpmt_set_launch(dpmt_ctx* ctx, int32_t launch);

/* Correlation tile configurations (output rows x 32 columns x filters per
 * workgroup, threads, one workgroup per tile or a resident grid striding the
 * tile list).  All accumulate each response in the same order, so results are
 * bitwise equal; only speed differs.  dpmt_tile_config_name returns a static
 * description, NULL outside [0, count). */
int32_t     dpmt_tile_config_count(void);
const char* dpmt_tile_config_name(int32_t config);
/* Select the configuration a mode uses (DPMT_E_UNSUPPORTED if the loaded
 * filters are too tall for it); dpmt_get_tile_config returns it (-1 on a bad
 * argument).  DPMT_CP_FP32 has one tile shape of its own: it accepts only
 * configuration 0, and dpmt_autotune times only that. */
dpmt_status dpmt_set_tile_config(dpmt_ctx* ctx, dpmt_mode mode, int32_t config);
int32_t     dpmt_get_tile_config(const dpmt_ctx* ctx, dpmt_mode mode);

/* Autotuner: runs the planned batch once per supported tile configuration as
 * a warm-up and then `reps` (1..1000) timed times with the batched strategy,
 * on hip_stream, waiting for each run; keeps the configuration with the
 * smallest median time for `mode`.  Same arguments and state rules as
 * dpmt_score_pyramid (its outputs are overwritten).  ms_out (host, may be
 * NULL) receives dpmt_tile_config_count() medians in milliseconds, -1 for
 * unsupported configurations; *best_out (may be NULL) the chosen index. */
dpmt_status dpmt_autotune(dpmt_ctx* ctx, dpmt_mode mode, const float* features_dev,
                          float* scores_dev, int16_t* offsets_dev, int32_t reps, float* ms_out,
                          int32_t* best_out, void* hip_stream);

const char* dpmt_status_string(dpmt_status s);
const char* dpmt_last_error(const dpmt_ctx* ctx);     /* detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* DPMT_H */
