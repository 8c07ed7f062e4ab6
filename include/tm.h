/*
 * tm.h - C ABI of the MI355X (gfx950) edge-orientation template matcher.
 *
 * The method is that of Le & Lin, "GPU-accelerated image alignment for object
 * detection in industrial applications" (arXiv 2112.05576), Sec. II: a model
 * image and a search image go through edge extraction and an image pyramid;
 * every pose (x, y, theta) of the top level is scored with the similarity
 * measure of Eq. (1) under the rigid projection of Eq. (2), each model point
 * taking its best vote over a neighbouring window (size 3 in the paper); the
 * best poses are then refined level by level down to the full image.
 *
 * Conventions for every call:
 *  - Device pointers ("_dev") are HIP device memory of the current device.
 *    Host pointers are plain host memory.  No call takes ownership of a
 *    caller buffer.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it and every call returns without waiting for the
 *    device, except tm_build_model (it waits once for the point counts) and
 *    the first call that has to grow an internal buffer (it waits before
 *    freeing the old one).  Inputs must stay valid until the stream has
 *    passed the call.
 *  - Every call returns a tm_status.  On failure nothing has been enqueued
 *    (validation happens first) and tm_last_error() describes the problem in
 *    the calling thread.  A failed HIP runtime call returns TM_EDEVICE.
 *  - A model may be used by any number of streams at once.  Its rotated-point
 *    tables are cached per (level, angle grid, scale grid); the first call
 *    with a new grid builds the table on its own stream and later calls on
 *    other streams wait for it (an event).  Under graph capture a table must
 *    already exist (run the call once before capturing).  A pyramid carries
 *    the scratch space of tm_detect / tm_refine, so one pyramid is used by one
 *    stream at a time.
 *  - Device memory of handles (models, pyramids, batches and their scratch)
 *    comes from the allocator registered with tm_set_allocator when the
 *    handle is created (default: hipMalloc / hipFree); a handle keeps that
 *    allocator for all its later allocations and frees.  Free a handle only
 *    after the streams that used it have passed their last use of it.
 *  - Result counts: a call that writes poses into a caller buffer of
 *    `capacity` entries writes to *n_out_dev the number of poses the method
 *    produced.  If that number exceeds `capacity`, only the first `capacity`
 *    of them (the best by the selection key, so the truncation is
 *    deterministic) are written: the result did not fit, which the caller
 *    reads as TM_ECAPACITY (the call itself returns before the device has
 *    counted, so this status travels in the count; the Python binding raises
 *    it).
 *
 * Image layout: uint8, row-major, `pitch` bytes between rows (pitch >= width).
 * Coordinates: x to the right, y down; the model's reference point is its
 * pixel (width/2, height/2) (integer division) at every pyramid level, and a
 * pose (x, y) places that point at search pixel (x, y) of the pose's level.
 */
#ifndef TM_H
#define TM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TM_OK = 0,
    TM_EINVAL = -1,    /* invalid argument (message says which)              */
    TM_ENOMEM = -2,    /* device or host allocation failed                   */
    TM_EDEVICE = -3,   /* a HIP runtime call failed                          */
    TM_ECAPACITY = -4  /* a result did not fit the caller's capacity        */
} tm_status;

typedef enum { TM_FP32 = 0, TM_FP16 = 1 } tm_precision;

/* Where the pyramid's gradients come from (Sec. II para. 2 names edge
 * extraction followed by the image pyramid; either order can be read there).
 * GREY: the grey image is reduced level by level and the Sobel pair is taken
 * on every level.  GRADIENT: the Sobel pair of the full image is taken once
 * and the gradient maps are reduced, each component of level l+1 being
 * floor((s + 2) / 4) of the 2x2 block sum s of level l. */
typedef enum { TM_PYR_GREY = 0, TM_PYR_GRADIENT = 1 } tm_pyr_source;

/* Which taps of a model point's window vote (Sec. II paras. 3-5, the
 * neighbouring search).  ALL: every tap, off the edge set and outside the
 * image with cosine 0.  EDGE: only taps on the edge set; a window without one
 * votes 0.  The centre-tap score S_1 is the same under both. */
typedef enum { TM_VOTE_ALL = 0, TM_VOTE_EDGE = 1 } tm_vote;

#define TM_MAX_LEVELS 8

/* Pyramid and edge parameters (Sec. II para. 2: edge detection threshold,
 * number of pyramid levels).  A pixel is an edge iff gx^2 + gy^2 >
 * floor(edge_thresh^2), gx and gy being the integer 3x3 Sobel responses
 * (zero on the one-pixel image frame); level l+1 is the 2x2 rounded mean of
 * level l, floor(w/2) x floor(h/2) (with `source` TM_PYR_GRADIENT the
 * gradient maps are reduced instead, see tm_pyr_source).  `precision`
 * selects how the search pyramid stores unit gradient directions (FP32, or
 * FP16 with FP32 accumulation); models ignore it. */
typedef struct {
    int32_t levels;       /* 1 .. TM_MAX_LEVELS                       */
    float edge_thresh;    /* >= 0, on the scale of the integer Sobel  */
    int32_t precision;    /* tm_precision                             */
    int32_t source;       /* tm_pyr_source (TM_PYR_GREY: the default) */
} tm_pyr_params;

/* Search parameters (Sec. II para. 2: step sizes in x, y and theta, the
 * neighbouring-search size) plus the multi-instance selection settings.
 * Angles: level l of an L-level search uses step theta_step_top_deg /
 * 2^(L-1-l) and angles theta_min_deg + k * step.  A range of 360 degrees or
 * more wraps (ceil(360/step) angles); a smaller range holds both end points
 * (floor(range/step + 1e-9) + 1 angles) and clamps.  The top level is
 * searched exhaustively on the grid x = i*step_x, y = j*step_y; each lower
 * level re-scores the 27 poses (2x+a, 2y+b, 2k+c), a, b, c in {-1, 0, 1}. */
typedef struct {
    int32_t step_x, step_y;       /* >= 1 pixels of the top level            */
    double theta_min_deg;
    double theta_range_deg;       /* > 0                                      */
    double theta_step_top_deg;    /* > 0, the angle step of the top level     */
    int32_t neighbourhood;        /* odd window side >= 1; the paper uses 3   */
    float min_score;              /* S_w floor for candidates and matches     */
    float nms_min_dist;           /* level-0 pixels; <= 0: half the model radius */
    int32_t max_candidates;       /* 1 .. 1024, kept after the top level      */
    int32_t max_matches;          /* >= 1, returned by tm_detect              */
    /* Similarity pose (the paper names other projection types than its rigid
     * Eq. (2)): p = sigma R(theta) t + u over the scales scale_min + j *
     * scale_step, j < scale_count.  The top level is searched over every
     * (angle, scale); lower levels refine (x, y, theta) at the chosen scale.
     * scale_count 1 with scale_min 1 is the rigid search. */
    double scale_min;             /* > 0 (1 for the rigid search)              */
    double scale_step;            /* >= 0                                      */
    int32_t scale_count;          /* 1 .. 64                                   */
    int32_t vote;                 /* tm_vote (TM_VOTE_ALL: the default)        */
} tm_search_params;

/* A pose with its scores.  (x, y) is in pixels of `level`; k indexes the
 * level's angle grid and theta_deg = theta_min + k * step is given for
 * convenience.  score_w is Eq. (1) with the neighbourhood vote, score_1 the
 * same with the centre tap only. */
typedef struct {
    int32_t x, y;
    int32_t k;
    int32_t level;
    float theta_deg;
    float score_w;
    float score_1;
    int32_t j;                    /* scale index (0 for the rigid search)     */
} tm_pose;

/* An arbitrary pose to score: integer translation, any angle. */
typedef struct {
    int32_t x, y;
    double theta_deg;
} tm_eval_pose;

/* A pose with continuous translation (pixels of its level) and angle, and
 * the (image, model) pair of a batch it belongs to (ignored outside one). */
typedef struct {
    float x, y, theta_deg;
    int32_t pair;
} tm_cont_pose;

typedef struct tm_model_s tm_model;
typedef struct tm_pyramid_s tm_pyramid;

/* Device-memory allocator for the handles (a caching allocator such as
 * torch's, say).  alloc returns `bytes` of device memory of the current
 * device, aligned to at least 256 bytes, or NULL on failure (the calling
 * entry point then returns TM_ENOMEM); `stream` is the stream of the call
 * that allocates (NULL when there is none).  free releases a block that
 * alloc returned; the library frees a block only after the stream it was
 * last used on has been synchronised, or at handle destruction (see the
 * conventions above).  ctx is passed through unchanged. */
typedef struct {
    void* (*alloc)(size_t bytes, void* ctx, void* stream);
    void (*free)(void* ptr, void* ctx, void* stream);
    void* ctx;
} tm_allocator;

/* Register the allocator used by handles created from now on (NULL, or
 * null function pointers: back to hipMalloc / hipFree).  Handles created
 * before keep the allocator they were created with.  TM_EINVAL if exactly
 * one of the two functions is null. */
tm_status tm_set_allocator(const tm_allocator* allocator);

/* Edge points of a model image on every pyramid level (Sec. II para. 2; the
 * points are the t_i of Eq. (2), row-major, relative to the reference pixel).
 * Waits on `stream` once to learn the point counts.  TM_EINVAL if the image
 * is smaller than 2^(levels-1) * 3 pixels a side or if a level has no edge
 * point.  The image is not retained. */
tm_status tm_build_model(const uint8_t* img_dev, int32_t width, int32_t height, int32_t pitch,
                         const tm_pyr_params* params, void* stream, tm_model** out);

/* Grey-level pyramid of a search image and its unit-gradient-direction field
 * on every level ((0, 0) off the edge set): Sec. II para. 2, edge extraction
 * (gradients and their magnitude against the threshold) and the image
 * pyramid whose top image the search starts from; Eq. (1) compares the
 * model's directions with this field.  Allocates the pyramid; the image is
 * copied, not retained.  TM_EINVAL if the image is smaller than
 * 2^(levels-1) * 3 pixels a side. */
tm_status tm_build_pyramid(const uint8_t* img_dev, int32_t width, int32_t height, int32_t pitch,
                           const tm_pyr_params* params, void* stream, tm_pyramid** out);

/* Rebuild an existing pyramid from a new image of the same size; allocates
 * nothing. */
tm_status tm_update_pyramid(tm_pyramid* pyr, const uint8_t* img_dev, int32_t pitch, void* stream);

/* Eq. (1) at n arbitrary poses of one level: scores_dev[2i] = S_w,
 * scores_dev[2i+1] = S_1 for poses_dev[i].  `neighbourhood` is the odd window
 * side (3 in the paper), `vote` a tm_vote.  Model points whose window falls
 * outside the image vote 0; the sum is divided by the model's point count at
 * that level. */
tm_status tm_score_poses(const tm_model* model, const tm_pyramid* pyr, int32_t level,
                         int32_t neighbourhood, int32_t vote, const tm_eval_pose* poses_dev, int32_t n,
                         float* scores_dev, void* stream);

/* Exhaustive search of one level (Sec. II para. 3, Fig. 2): for every
 * translation of the step grid, the best angle of the level's grid by the key
 * (S_w desc, S_1 desc, k asc).  Outputs are [gh][gw] arrays with
 * gw = ceil(w_level/step_x), gh = ceil(h_level/step_y). */
tm_status tm_score_map(const tm_model* model, tm_pyramid* pyr, int32_t level,
                       const tm_search_params* params, float* sw_dev, float* s1_dev, int32_t* k_dev,
                       void* stream);

/* Candidate selection on a score map of `level` (layout as tm_score_map).
 * Sec. II para. 3 records a pose whenever its score is better than the best
 * so far, i.e. it keeps the single best pose; for several instances this is
 * generalised to: grid points with S_w >= min_score whose key (S_w desc,
 * S_1 desc, x asc, y asc) beats all 8 grid neighbours, sorted by the key,
 * thinned greedily so that accepted poses are >= dmin apart in level-0 pixels
 * (distance scaled by 2^level), at most `capacity` (1..1024, the method's cap
 * on candidates, like max_candidates in a detection: reaching it is not an
 * overflow).  Writes the poses and their count (device int).  Inputs: device
 * maps of gw x gh (sw, s1 float; k int32); outputs: device buffers.  Used
 * inside tm_detect; exported so that it can be run on a given map. */
tm_status tm_select(const float* sw_dev, const float* s1_dev, const int32_t* k_dev, int32_t gw, int32_t gh,
                    int32_t step_x, int32_t step_y, int32_t level, float min_score, float dmin,
                    tm_pose* out_dev, int32_t capacity, int32_t* n_out_dev, void* stream);

/* Full detection (Sec. II): exhaustive search of the top level, candidate
 * selection (at most max_candidates), refinement down to level 0, then the
 * final selection: candidates with S_w >= min_score, key order, greedy
 * suppression within nms_min_dist, at most max_matches.  *n_out_dev gets
 * their number and out_dev (capacity entries) the first min(number,
 * capacity) of them at level 0; a number above capacity is the TM_ECAPACITY
 * case of the conventions above. */
tm_status tm_detect(const tm_model* model, tm_pyramid* pyr, const tm_search_params* params,
                    tm_pose* out_dev, int32_t capacity, int32_t* n_out_dev, void* stream);

/* Bytes of the static device array behind tm_detect_static (one per GPU). */
#define TM_STATIC_SCRATCH_BYTES (64u << 20)

/* tm_detect for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same detection, with the same results as tm_detect, but every scratch
 * buffer (the pair descriptor, the top level's rotated table, rebuilt on
 * each call, the search partials and score map, the selection and
 * refinement scratch) lives in a static device array of
 * TM_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, instead of the pyramid's workspace and the model's
 * table cache.  Allocates nothing (no hipMalloc, no registered allocator)
 * and reads the model and pyramid without changing them.  Returns
 * TM_ECAPACITY, with nothing enqueued, if the detection needs more than
 * TM_STATIC_SCRATCH_BYTES (large top levels, many angles); otherwise the
 * arguments and the result count are those of tm_detect.  Every call on one
 * GPU shares that GPU's array, which keeps the last call's contents: calls
 * that overlap on one GPU (on other streams or threads) race, so serialise
 * them. */
tm_status tm_detect_static(const tm_model* model, const tm_pyramid* pyr, const tm_search_params* params,
                           tm_pose* out_dev, int32_t capacity, int32_t* n_out_dev, void* stream);

/* Coarse-to-fine refinement of n poses of level `from_level` (x, y, k on
 * that level's grid) down to level 0, in place (Sec. II para. 2: the search
 * begins at the top image of the pyramid and is carried down to the full image;
 * the paper gives no neighbourhood for the step, this uses the 3 x 3 x 3 one
 * around the doubled pose): at each level below, the pose is replaced by the
 * best (by the selection key) of the 27 poses (2x+a, 2y+b, 2k+c),
 * a, b, c in {-1, 0, 1}, inside the level image, scored with Eq. (1) and the
 * neighbouring window.  poses_dev: n device tm_pose records, read and
 * written; poses must lie inside their level.  No selection is applied. */
tm_status tm_refine(const tm_model* model, tm_pyramid* pyr, const tm_search_params* params, int32_t from_level,
                    tm_pose* poses_dev, int32_t n, void* stream);

/* --- continuous score (differentiable; an extension beside Eq. (1)) ---- */

/* S_c = (1/n) sum_i r_i . B(R(theta) t_i + u): the model's rotated
 * directions against the bilinearly interpolated direction field of `level`
 * (zero off the edge set and outside the image), no window, no rounding.
 * scores_dev[i] for poses_dev[i]; FP32. */
tm_status tm_cont_score(const tm_model* model, tm_pyramid* pyr, int32_t level, const tm_cont_pose* poses_dev,
                        int32_t n, float* scores_dev, void* stream);

/* Backward of tm_cont_score: grad_poses_dev[3i..3i+2] = grad_scores_dev[i] *
 * dS_c/d(x, y, theta_deg) of pose i (grad_scores_dev NULL: ones).  The
 * derivative is that of the bilinear patch (pixel cell) containing each
 * projected point. */
tm_status tm_cont_score_backward(const tm_model* model, tm_pyramid* pyr, int32_t level,
                                 const tm_cont_pose* poses_dev, int32_t n, const float* grad_scores_dev,
                                 float* grad_poses_dev, void* stream);

/* Line search in FP64: for each pose i, S_c evaluated in double precision at
 * pose + alphas[j] * dirs_dev[3i..3i+2] rounded to the FP32 pose record,
 * j < n_alphas (host array, 1 to 16 finite values); the pose moves to the
 * best (ties: the earlier step) and scores_dev[i] (may be NULL) receives
 * that score.  Uses the pyramid's scratch (8 bytes per evaluation). */
tm_status tm_cont_line_search(const tm_model* model, tm_pyramid* pyr, int32_t level, tm_cont_pose* poses_dev,
                              const float* dirs_dev, int32_t n, const double* alphas, int32_t n_alphas,
                              float* scores_dev, void* stream);

/* --- batches ------------------------------------------------------------ */

/* A batch binds n_images device images (each width x height, `pitch` bytes
 * per row) and n_models models to output buffers, for the detection of
 * every model in every image (Sec. II applied pair by pair).  Pair
 * p = image * n_models + model writes its matches (at most max_matches) to
 * out_dev[p * capacity ...] and their number to n_out_dev[p]; a number above
 * capacity is the TM_ECAPACITY case of the conventions above (the first
 * capacity matches by key are written).
 * Creation allocates the pyramids, the rotated tables of the top level and
 * all scratch, and waits for the uploads; models must outlive the batch (their
 * points are read, their table cache is not used).  At most 65535 pairs.
 * The exhaustive search runs over a work list fixed here: each pair's
 * blocks, heaviest models first, dealt to the eight XCDs in equal-cost
 * contiguous runs, so that uneven pairs do not leave a tail. */
typedef struct tm_batch_s tm_batch;
tm_status tm_batch_create(const tm_model* const* models, int32_t n_models, const uint8_t* const* images_dev,
                          const int32_t* widths, const int32_t* heights, const int32_t* pitches, int32_t n_images,
                          const tm_pyr_params* pyr_params, const tm_search_params* params, tm_pose* out_dev,
                          int32_t capacity, int32_t* n_out_dev, void* stream, tm_batch** out);

/* Enqueue the whole batch: pyramids and direction fields of every bound image
 * (read at execution time, so new contents in the same buffers are picked
 * up), then the exhaustive search, selection, refinement and final selection
 * of every pair, each stage one launch over all pairs.  Allocates nothing and
 * never waits, so it can be captured in a graph. */
tm_status tm_batch_run(tm_batch* batch, void* stream);

/* As tm_batch_run, as one graph launch: the first call captures the batch's
 * launches into a HIP graph (on a private stream, without running them) and
 * keeps it with the batch; every call then launches that graph on `stream`.
 * Search-kernel timing (tm_timing_enable) does not apply to graph launches. */
tm_status tm_batch_run_graph(tm_batch* batch, void* stream);

/* Autotuner of a batch's exhaustive search (the search is 99 % of the work;
 * its schedule is what the tuner picks).  The schedule has three
 * dimensions: the instruction-level variant of the search kernel (0..5), the
 * waves sharing an angle chunk (2, 4, 8, 16; a workgroup stages one field
 * tile for them) and the angle chunk (how many angles one workgroup scores:
 * the batch holds up to four times its planned number of chunks, at most
 * 12).  First every (variant, waves) form that fits in LDS is timed on the
 * search alone at the planned chunking, `iterations` launches each, twice
 * over (a form's time is the smaller of its two rounds); then the two
 * fastest forms are timed at every chunking.  With a partner (a batch of the
 * same shape, run on its own partner_stream) the second stage times the
 * pipelined step of the two batches as graph launches alternating on the two
 * streams, which is what a caller keeping two batches in flight runs, and
 * both batches end with the choice; without one it times the search alone.
 * Runs the pyramid stage first; waits for the device.  All schedules give
 * bit-identical results; tuning changes only time.  variant_out, waves_out,
 * chunk_out (angles per chunk), us_out (each may be NULL): the choice and its
 * time (per step with a partner, per search launch without).  For a batch on
 * the generic search there is nothing to choose: -1, 0, 0, 0. */
tm_status tm_batch_tune(tm_batch* batch, tm_batch* partner, int32_t iterations, void* stream, void* partner_stream,
                        int32_t* variant_out, int32_t* waves_out, int32_t* chunk_out, float* us_out);

/* Use the given schedule of the search for the batch's later runs (one
 * reported by tm_batch_tune or tm_batch_search_form of a batch of the same
 * shape, say): TM_EINVAL if it does not apply (variant 0..5, 1..16 waves
 * sharing a chunk, within LDS; the edge-taps vote has one variant per
 * precision; chunk: angles per chunk, 0 keeps the current chunking, and the
 * chunks must not outnumber what the batch holds; -1 is accepted, and
 * changes nothing, for a batch on the generic search).  Results do not depend
 * on the schedule.  Waits for the batch's last run; a captured graph is
 * discarded and captured again by the next tm_batch_run_graph. */
tm_status tm_batch_set_form(tm_batch* batch, int32_t variant, int32_t waves, int32_t chunk);

/* The schedule of the batch's exhaustive search now in use (default or
 * tuned): kernel variant, waves sharing an angle chunk and angles per chunk
 * (chunk may be NULL; -1, 0, 0 for the generic search). */
tm_status tm_batch_search_form(const tm_batch* batch, int32_t* variant, int32_t* waves, int32_t* chunk);

/* Launch shape of the batch's search kernel in its current schedule:
 * workgroups per launch and threads per workgroup (inspection: matches a
 * profiler's dispatch records to a schedule). */
tm_status tm_batch_search_launch(const tm_batch* batch, int32_t* workgroups, int32_t* threads);

/* The continuous score, its backward and the FP64 line search (as
 * tm_cont_score, tm_cont_score_backward and tm_cont_line_search) over the
 * pairs of a batch, against the fields its last run built: pose.pair names
 * the pair (image * n_models + model); a pose naming no pair of the batch
 * gets NaN results (the line search leaves it where it is).  The line search
 * keeps its scratch with the batch (allocated, or grown, on first need). */
tm_status tm_batch_cont_score(tm_batch* batch, int32_t level, const tm_cont_pose* poses_dev, int32_t n,
                              float* scores_dev, void* stream);
tm_status tm_batch_cont_score_backward(tm_batch* batch, int32_t level, const tm_cont_pose* poses_dev, int32_t n,
                                       const float* grad_scores_dev, float* grad_poses_dev, void* stream);
tm_status tm_batch_cont_line_search(tm_batch* batch, int32_t level, tm_cont_pose* poses_dev, const float* dirs_dev,
                                    int32_t n, const double* alphas, int32_t n_alphas, float* scores_dev,
                                    void* stream);

/* The pyramid the batch built for one image (owned by the batch).  An FP16
 * batch keeps FP16 directions at its searched (top) level only: below it the
 * pyramid holds the uint8 levels and the FP32 directions its refinement
 * reads, so tm_pyramid_level gives a null field there and tm_pyramid_read
 * (field), tm_score_poses and tm_score_map of those levels fail with
 * TM_EINVAL. */
tm_status tm_batch_pyramid(const tm_batch* batch, int32_t image, const tm_pyramid** out);

void tm_batch_free(tm_batch* batch);

/* --- inspection (tests, tools) ------------------------------------------ */

/* Level geometry of a model: size of the level image and point count. */
tm_status tm_model_level_info(const tm_model* model, int32_t level, int32_t* width, int32_t* height,
                              int32_t* n_points);

/* Copy a model level's points to device buffers: t_dev[2i..2i+1] = t_i
 * (int32), g_dev[2i..2i+1] = the integer Sobel gradient at the point. */
tm_status tm_model_points(const tm_model* model, int32_t level, int32_t* t_dev, int32_t* g_dev,
                          void* stream);

/* Rotated model table of a level for angles theta_min + k * step, k < K:
 * q_dev[(k*n + i)*2 ..] = round(R t_i) (int32 pairs), r_dev[...] = R d_i
 * (float pairs), with the rounding rule floor(v + 0.5 + 1e-9) in FP64. */
tm_status tm_model_table(const tm_model* model, int32_t level, double theta_min, double step, int32_t K,
                         int32_t* q_dev, float* r_dev, void* stream);

/* Level geometry and device storage of a pyramid: the uint8 image (row-major,
 * pitch = width) and the direction field (pairs of float, or of half for
 * TM_FP16, row-major).  The pointers stay owned by the pyramid. */
tm_status tm_pyramid_level(const tm_pyramid* pyr, int32_t level, int32_t* width, int32_t* height,
                           const uint8_t** img_dev, const void** field_dev, int32_t* precision);

/* Copy a pyramid level into caller device buffers (either may be NULL):
 * img_dev gets width*height bytes, field_dev width*height pairs (float, or
 * half for TM_FP16). */
tm_status tm_pyramid_read(const tm_pyramid* pyr, int32_t level, uint8_t* img_dev, void* field_dev, void* stream);

/* Stage timing.  While enabled, tm_detect and tm_score_map record a pair of
 * HIP events around the exhaustive-search kernel on the call's stream.
 * tm_timing_read waits for the recorded events, returns the summed kernel
 * time in milliseconds and the number of launches, and clears the record. */
tm_status tm_timing_enable(int32_t on);
tm_status tm_timing_read(double* dense_ms, int32_t* launches);

/* Ceiling probes for the roofline of the exhaustive search (measurement
 * infrastructure, not part of the method): one launch that runs a single
 * instruction mix of the search at full occupancy, enqueued on `stream`; the
 * caller times it (events around the call) and divides *work_out by the time.
 *  kind 0: the search's per-point arithmetic (10 v_dot2_f32_f16, 8 v_max3_f32,
 *          16 DPP maxima, 8 sums): *work_out = wave-level VALU instructions;
 *  kind 1: independent v_add_f32: *work_out = wave-level VALU instructions;
 *  kind 2: the search's LDS reads (10 rows of a strip a lane, 4 bytes each,
 *          at a moving wave-uniform offset): *work_out = bytes read;
 *  kind 3: streaming copy of the first half of buf_dev into the second:
 *          *work_out = bytes read plus written (HBM stream);
 *  kinds 4, 5, 6: one instruction class of the mix at a time (v_dot2_f32_f16,
 *          DPP v_max_f32, v_max3_f32): *work_out = wave-level VALU instructions.
 * iterations (1 .. 10^6) sets the length of kinds 0-2; buf_dev is device
 * memory of buf_bytes bytes (>= 256; kinds 0-2 only write it if a result
 * that never occurs comes out).  TM_EINVAL on a bad kind or size. */
tm_status tm_probe(int32_t kind, int32_t iterations, void* buf_dev, int64_t buf_bytes, void* stream,
                   double* work_out);

void tm_model_free(tm_model* model);
void tm_pyramid_free(tm_pyramid* pyr);

/* Description of the last failure in the calling thread ("" if none). */
const char* tm_last_error(void);

/* Library version string. */
const char* tm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TM_H */
