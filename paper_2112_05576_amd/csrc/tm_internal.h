// Internal declarations of the HIP template matcher: handle layouts, table
// records and kernel launchers.  Host code only includes this through the
// .hip translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "../../include/tm.h"

namespace tmk {

constexpr int kMaxLevels = TM_MAX_LEVELS;
// The refinement's sums of one candidate and level: for each of its 3 angles,
// the 18 sums (9 windowed, 9 centre) of each of the kRefineWaves waves that
// share the angle's points; a sum over the angle's points is the waves' sums
// added in wave order.
constexpr int kRefineWaves = 4;
constexpr int kPartPerCand = 3 * kRefineWaves * 18;

// One model edge point: offset t from the level's reference pixel and the
// integer Sobel gradient (the unit direction d = g/|g| is formed in FP64
// where a table is built).
struct ModelPoint {
    int16_t tx, ty, gx, gy;
};

// One entry of a rotated model table (Eq. 2 applied to a point at one angle):
// q = round(R t) with the FP64 rule floor(v + 0.5 + 1e-9), r = R d as FP32 and
// as packed FP16.  16 bytes so that a wave reads one entry with one scalar
// load.
struct alignas(16) TabEntry {
    int16_t qx, qy;
    float rx, ry;
    uint32_t rh;  // half2 (rx, ry)
};

struct PyrLevel {
    int w, h;
    uint8_t* img;   // w*h bytes, row-major
    void* field;    // w*h float2 (FP32) or half2 (FP16), row-major: the storage the searches read
    void* field32;  // w*h float2: the FP32 field (the same buffer as `field` in an FP32 pyramid; an FP16
                    // pyramid keeps this twin for the decisions taken after its FP16 search)
    uint32_t* grad; // gradient-map pyramid only: w*h packed int16 pairs (gx low, gy high); else null
};

struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Device memory through the allocator a handle was created with (null
// functions: hipMalloc / hipFree).
hipError_t dev_alloc(const tm_allocator& a, void** p, size_t bytes, hipStream_t s);
void dev_free(const tm_allocator& a, void* p, hipStream_t s);

}  // namespace tmk

struct tm_pyramid_s {
    tm_allocator alloc = {};  // allocator of this pyramid's memory
    int L = 0;
    int precision = TM_FP32;
    int source = TM_PYR_GREY;
    float tau = 0.f;
    long long T2 = 0;
    int dev = 0;
    tmk::PyrLevel lv[tmk::kMaxLevels] = {};
    void* block = nullptr;  // single allocation holding all levels
    tmk::Workspace ws;       // scratch of detect / refine / score_map
    bool desc_valid = false;  // ws starts with a device copy of last_desc
    unsigned char last_desc[1024];
};

struct tm_model_level {
    int w = 0, h = 0, n = 0, n_pad = 0;
    int radius2 = 0;    // max |t|^2
    int rad = 0;        // bound on |q| components over all angles
    tmk::ModelPoint* pts = nullptr;  // device, n entries
    double2* dir = nullptr;          // device, n FP64 unit directions g/|g|
};

// One rotated table of a model level for one angle and scale grid.
struct tm_rot_table {
    int level = -1;
    double theta_min = 0, step = 0;
    int K = 0;
    int S = 0;
    double sigma_min = 0, sigma_step = 0;
    tmk::TabEntry* tab = nullptr;  // device, K * S * n_pad entries
    hipEvent_t ready = nullptr;    // recorded after the table's kernel
    hipStream_t stream = nullptr;  // stream the table was built on
};

struct tm_model_s {
    tm_allocator alloc = {};  // allocator of this model's memory
    int L = 0;
    float tau = 0.f;
    int source = TM_PYR_GREY;
    int dev = 0;
    tm_model_level lv[tmk::kMaxLevels];
    std::mutex mu;                       // guards `tables`
    std::vector<tm_rot_table> tables;  // one per (level, grid), kept until the model is freed
};

namespace tmk {

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return the hipGetLastError() status.

// Arguments of the pyramid kernels for one image (by value for one image, in
// device memory for a batch).
struct PyrBuildArg {
    const uint8_t* src;          // caller's image (level 0 source)
    int pitch;
    int L;
    uint8_t* img[kMaxLevels];    // level images
    int w[kMaxLevels];
    int h[kMaxLevels];
};

struct FieldsArg {
    const uint8_t* img[kMaxLevels];
    uint32_t* grad[kMaxLevels];  // gradient-map pyramid (all null: gradients of each grey level)
    void* field[kMaxLevels];
    void* field32[kMaxLevels];   // FP16 pyramids: the FP32 twin, written beside the half2 field (else null)
    int w[kMaxLevels];
    int h[kMaxLevels];
    int block0[kMaxLevels + 1];  // first workgroup of each level
    int L;
    int precision;
    long long T2;
};

PyrBuildArg pyr_build_arg(const uint8_t* src, int src_pitch, const PyrLevel* lv, int L);
FieldsArg fields_arg(const PyrLevel* lv, int L, long long T2, int precision);
// Pyramids and fields of n_images images in one pass (pb, fa: device arrays);
// level_w/level_h: largest level sizes over the images; gradient: build the
// gradient-map pyramids (fa[i].grad) before the fields.
hipError_t launch_pyramids_batch(const PyrBuildArg* pb, const FieldsArg* fa, int n_images, int L, int max_w,
                                 int max_h, int max_field_blocks, const int* level_w, const int* level_h,
                                 bool gradient, hipStream_t s);

// Level-0 copy (pitched source) and uint8 levels base+1 .. top.
hipError_t launch_pyr_build(const uint8_t* src, int src_pitch, const PyrLevel* lv, int L, hipStream_t s);
// Gradient-map pyramid: the Sobel pair of level 0's image into grad[0],
// then floored 2x2 means level by level (levels with grad set).
hipError_t launch_grad_pyramid(const PyrLevel* lv, int L, hipStream_t s);
// Unit direction fields of levels 0 .. L-1 (FP32 or FP16), from lv[l].grad
// where set, else from the Sobel pair of the level's image.
hipError_t launch_sobel_fields(const PyrLevel* lv, int L, long long T2, int precision, hipStream_t s);
// Row-major edge points of each model level into pts[l] (capacity w*h),
// counts into counts[l].
hipError_t launch_model_points(const PyrLevel* lv, int L, long long T2, ModelPoint* const* pts, int* counts,
                               hipStream_t s);
// Projected table of one level for angles theta_min + k*step, k < K, and
// scales sigma_min + j*sigma_step, j < S: entry [j*K + k][i].
hipError_t launch_tables(const ModelPoint* pts, int n, int n_pad, double theta_min, double step, int K,
                         double sigma_min, double sigma_step, int S, TabEntry* tab, hipStream_t s);
// FP64 unit direction g/|g| of every point (the arithmetic of the projection).
hipError_t launch_unit_dirs(const ModelPoint* pts, int n, double2* dir, hipStream_t s);
// Expand a table into plain int32 q pairs and float r pairs.
hipError_t launch_table_export(const TabEntry* tab, int n, int n_pad, int K, int32_t* q, float* r, hipStream_t s);

// One (image, model) pair of a detection: the image's pyramid levels, the
// model's levels, the rotated table of the searched level, and the pair's
// scratch and result buffers.  Lives in device memory; kernels take the pair
// from blockIdx.y.
struct PairDesc {
    const void* field[kMaxLevels];   // FP32 direction field per level (refinement, re-scoring)
    const void* sfield;              // field the exhaustive search reads (the searched level, storage precision)
    int W[kMaxLevels], H[kMaxLevels];
    const ModelPoint* pts[kMaxLevels];
    const double2* dir[kMaxLevels];  // FP64 unit directions of the points
    int n[kMaxLevels];
    const TabEntry* tab;             // rotated table of the searched level, [K][n_pad]
    int n_pad, rad;                  // table padding; bound on |q| at the searched level
    int gw, gh;                      // translation grid of the searched level
    int tiles_x, tiles_y;            // search tiles along the lanes and the strips (fast path)
    float dmin;                      // suppression distance, level-0 pixels
    float* pw;                       // chunk partials [C][gh][gw]: best S_w,
    float* p1;                       //   S_1,
    int32_t* pk;                     //   angle; a certified (screen) search also keeps
    float* p2;                       //   the runner-up's S_w,
    int32_t* pk2;                    //   its angle,
    float* p3;                       //   and the best S_w of the chunk's remaining angles
    float* mw;                       // best angle per translation [gh][gw]: S_w,
    float* m1;                       //   S_1,
    int32_t* mk;                     //   angle; a certified search also keeps
    float* m2;                       //   the runner-up's S_w,
    int32_t* mk2;                    //   its angle,
    float* m3;                       //   and the best S_w of the remaining angles
    float* sel;                      // selection scratch, select_scratch_bytes(gw*gh)
    tm_pose* cand;                   // candidates [max_cand] (refined in place)
    int32_t* ncand;                  // their count (device); null: max_cand
    tm_pose* ctr[2];                 // refinement centres [max_cand]
    float* part[kMaxLevels];         // refinement sums [max_cand][3][kRefineWaves][18]
    int rad_l[kMaxLevels];           // bound on |q| components at each level
    int rtile[kMaxLevels];           // 1: level refined by the staged kernel (partials: one chunk)
    void* pfield;                    // generic search: the searched field with a zero border
    int pW, pH, pad;                 //   its size and border width
    tm_pose* out;                    // results [capacity]
    int32_t* n_out;                  // their count
};

// Settings shared by every pair of a launch.
struct SearchDesc {
    int L;                      // pyramid levels
    int level;                  // level searched exhaustively (or selected / refined from)
    int K[kMaxLevels];          // angles per level
    double step[kMaxLevels];    // angle step per level
    double theta_min;
    int full, win, sx, sy, precision;
    int vote;                   // tm_vote: which taps of a window vote
    float min_score;
    int max_cand;               // candidates kept after the searched level
    int capacity;               // poses the caller's result buffer holds
    int max_matches;            // final matches kept (the method's cap)
    int S;                      // scales (1: rigid)
    double sigma_min, sigma_step;
    int screen;                 // FP16 detection: the search is a screen whose decisions are certified
};

// Poses per translation at the searched level: angles x scales, indexed
// m = j * K + k (scale-major).
inline int poses_per_translation(const SearchDesc& s) { return s.K[s.level] * s.S; }

// Launch plan of the exhaustive search, common to all pairs.
struct DensePlan {
    bool fast;
    int prec;                   // precision of the searched field
    bool screen;                // FP16 screen of a certified detection (no S_1; runner-up kept)
    int vote;                   // tm_vote (the edge-taps reading has one kernel form)
    int variant;                // search kernel form (k_dense_fast VAR)
    int tr;                     // 1: lanes along y, strips along x (FastArgs.tr)
    int G, R, LC, WY, WA;
    int A, C;                   // angles per workgroup, chunks of angles
    size_t lds;
    size_t tile_lds;            // the field tile's share of lds
    int max_blocks;             // workgroups of the largest pair (fast path)
    int max_np;                 // translations of the largest pair
    int max_rad;                // largest bound on |q| components over the pairs
    const int2* work = nullptr; // optional device work list (fast path, build_work)
    int n_work = 0;
    // generic path: bytes per field pixel, window half-width, and the largest
    // zero-bordered field copy over the pairs (pixels)
    int px_bytes = 0, win_h = 0;
    long long max_pad_px = 0;
};

// The searched level of one pair, for planning.
struct PairGeom {
    int W, H, gw, gh, rad, n;
};

DensePlan plan_dense(const SearchDesc& s, const PairGeom* g, int npairs);
// Another form of a fast plan with the same tiles and angle chunks (so the
// same scratch and work list): kernel variant and waves sharing a chunk.
// false if the plan is not the fast path or the form does not fit.
bool retune_dense(DensePlan& p, int variant, int WA);
// Another angle chunking of a fast plan (A angles a chunk, rounded up to a
// multiple of 4; the same tiles and form): chunks and workgroups follow.
bool rechunk_dense(DensePlan& p, const SearchDesc& s, const PairGeom* g, int npairs, int A);
// The distinct chunk sizes (angles) that give at most c_max chunks.
std::vector<int> chunk_candidates(const DensePlan& p, const SearchDesc& s, int c_max);
// Tile counts of a pair under a plan (fast path).
void plan_tiles(const DensePlan& p, const PairGeom& g, int* tiles_x, int* tiles_y);
size_t dense_partials_bytes(const DensePlan& p, int np);
// Work list of the fast search over many pairs: the blocks binned onto the
// eight XCDs to equal cost, heaviest first (longest processing time), pairs
// kept contiguous within a bin for L2 reuse of their tables; entry b is run
// by workgroup b, (-1, 0) entries pad the bins to equal length.  Empty when
// the plan is not the fast path; false if the list failed its own check
// (every block of every pair exactly once).
bool build_work(const DensePlan& p, const PairGeom* g, int npairs, std::vector<int2>& out);
size_t select_scratch_bytes(int np);
// Refinement plan of a launch.  staged: pairs whose level block fits
// (PairDesc.rtile) are refined by the staged kernel, the others by gathers;
// otherwise all by gathers (both give bit-identical sums; staging pays off
// once a launch holds many candidates).  Per level: whether any pair is
// refined by gathers, and the largest staged block (0: none).
struct RefinePlan {
    int staged;
    int gather[kMaxLevels];
    int tile_bytes[kMaxLevels];
};
// LDS bytes of the staged field block of a level (side 2 rad + 5) and
// whether the level is refined from it (window 3 and at most 128 KB).
size_t refine_tile_bytes(int rad, int precision);
bool refine_tile_fits(int rad, int precision, int win);

// Kernel attributes of the plan's search kernel (call before capturing it).
hipError_t prepare_dense(const SearchDesc& s, const DensePlan& p);
// Exhaustive search of s.level for every pair: pair.mw/m1/mk.  ev0 / ev1
// (optional) are recorded around the search kernel only.  cert_count
// (optional, a certified search): the certification's list counter, cleared
// by the search's last kernel so that launch_certify needs no kernel for it.
hipError_t launch_dense(const SearchDesc& s, const DensePlan& p, const PairDesc* d, int npairs, hipStream_t st,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int* cert_count = nullptr);
// Certification of an FP16 search (see k_score.hip): translations whose
// FP32 scores could decide the candidate selection are re-scored in FP32 from
// the FP32 twin, with the FP32 search's arithmetic, over the angles their FP16
// scores leave open, and the map takes those values.  Buffers (device): a
// counter and a list with room for every translation of every pair.
struct CertBufs {
    int* count;       // entries in `list`
    int4* list;       // (pair, translation, angle a, angle b or -1), or (-1 - pair, translation,
                      // chunk mask low, high): the angles to score in FP32
    int cap;          // entries the list holds (every translation of every pair)
};
size_t cert_bytes(int total_np);
CertBufs cert_bufs(void* base, int total_np);
// Enqueues: the counter cleared (a kernel, not a memset) unless the search
// before it cleared it (count_cleared: launch_dense had cb.count), the
// flagging of the translations, and the re-scoring kernel.
hipError_t launch_certify(const SearchDesc& s, const DensePlan& p, const PairDesc* d, int npairs, const CertBufs& cb,
                          hipStream_t st, bool count_cleared = false);

// Candidates of every pair from its map: pair.cand / ncand (<= s.max_cand).
hipError_t launch_select(const SearchDesc& s, const PairDesc* d, int npairs, int max_np, hipStream_t st);
// Refine pair.cand (poses of level from_level) down to level 0, in place.
// pick: end with the pick of the level-0 poses into pair.cand; without it the
// level-0 sums and centres are left for launch_final (centre buffer
// from_level % 2).
hipError_t launch_refine(const SearchDesc& s, const PairDesc* d, int npairs, int from_level, const RefinePlan& rp,
                         hipStream_t st, bool pick = true);
// Kernel attributes of the staged refinement (call before capturing it).
hipError_t prepare_refine();
// Final selection of every pair: pair.cand -> pair.out / n_out.
// out / n_out (one pair only, optional): write there instead of the pair's
// own result buffers, so a descriptor need not change with the caller's output.
// pick >= 0: the candidates are the best of their 27 level-0 sums, centres in
// pair.ctr[pick] (a refinement launched without its own pick).
hipError_t launch_final(const SearchDesc& s, const PairDesc* d, int npairs, hipStream_t st, tm_pose* out = nullptr,
                        int32_t* n_out = nullptr, int pick = -1);

// Continuous score (forward) or its backward of n poses; d: descriptor array
// of npairs entries (batched: pose.pair selects, else descriptor 0).
hipError_t launch_cont(const PairDesc* d, int batched, int npairs, int level, int precision, const tm_cont_pose* poses,
                       int n, const float* gin, float* out, bool backward, hipStream_t s);
size_t line_search_scratch_bytes(int n, int n_alpha);
hipError_t launch_line_search(const PairDesc* d, int batched, int npairs, int level, int precision,
                              tm_cont_pose* poses, const float* dirs, int n, const double* alphas, int n_alpha,
                              float* scores, double* scratch, hipStream_t s);

// Ceiling probes (k_roof.hip): kind 0 the search's VALU mix, 1 plain VALU
// adds, 2 LDS reads of the search's pattern, 3 an HBM copy within buf; work:
// VALU instructions (waves), LDS bytes, or HBM bytes enqueued.
hipError_t launch_probe(int kind, int iters, void* buf, long long buf_bytes, hipStream_t s, double* work);

// One wave per pose: S_w and S_1 of arbitrary poses.
hipError_t launch_sparse(const void* field, int W, int H, int precision, const ModelPoint* pts, int n, int win,
                         int vote, const tm_eval_pose* poses, int np, float* scores, hipStream_t s);

}  // namespace tmk
