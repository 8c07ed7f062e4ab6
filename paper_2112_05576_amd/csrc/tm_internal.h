// Internal declarations of the HIP template matcher: handle layouts, table
// records and kernel launchers.  Host code only includes this through the
// .hip translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "../../include/tm.h"

namespace tmk {

constexpr int kMaxLevels = TM_MAX_LEVELS;

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
    void* field;    // w*h float2 (FP32) or half2 (FP16), row-major
};

struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace tmk

struct tm_pyramid_s {
    int L = 0;
    int precision = TM_FP32;
    float tau = 0.f;
    long long T2 = 0;
    int dev = 0;
    tmk::PyrLevel lv[tmk::kMaxLevels] = {};
    void* block = nullptr;  // single allocation holding all levels
    tmk::Workspace ws;       // scratch of detect / refine / score_map
};

struct tm_model_level {
    int w = 0, h = 0, n = 0, n_pad = 0;
    int radius2 = 0;    // max |t|^2
    int rad = 0;        // bound on |q| components over all angles
    tmk::ModelPoint* pts = nullptr;  // device, n entries
};

struct tm_model_table_cache {
    int level = -1;
    double theta_min = 0, step = 0;
    int K = 0;
    tmk::TabEntry* tab = nullptr;  // device, K * n_pad entries
    size_t cap = 0;               // entries allocated
};

struct tm_model_s {
    int L = 0;
    float tau = 0.f;
    int dev = 0;
    tm_model_level lv[tmk::kMaxLevels];
    tm_model_table_cache cache;
};

namespace tmk {

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return the hipGetLastError() status.

// Level-0 copy (pitched source) and uint8 levels base+1 .. top.
hipError_t launch_pyr_build(const uint8_t* src, int src_pitch, const PyrLevel* lv, int L, hipStream_t s);
// Unit direction fields of levels 0 .. L-1 (FP32 or FP16).
hipError_t launch_sobel_fields(const PyrLevel* lv, int L, long long T2, int precision, hipStream_t s);
// Row-major edge points of each model level into pts[l] (capacity w*h),
// counts into counts[l].
hipError_t launch_model_points(const PyrLevel* lv, int L, long long T2, ModelPoint* const* pts, int* counts,
                               hipStream_t s);
// Rotated table of one level for angles theta_min + k*step, k < K.
hipError_t launch_tables(const ModelPoint* pts, int n, int n_pad, double theta_min, double step, int K,
                         TabEntry* tab, hipStream_t s);
// Expand a table into plain int32 q pairs and float r pairs.
hipError_t launch_table_export(const TabEntry* tab, int n, int n_pad, int K, int32_t* q, float* r, hipStream_t s);

struct DenseGeom {
    const void* field;
    int W, H;             // level size
    int precision;
    const TabEntry* tab;  // [K][n_pad]
    int n, n_pad, K;
    int sx, sy, win;      // step grid, window side
    int rad;              // |q| bound
    int gw, gh;           // grid size
};

// Exhaustive search of one level: best (S_w, S_1, k) per grid translation.
// Uses ws (device scratch) of at least dense_workspace_bytes(g) bytes.
size_t dense_workspace_bytes(const DenseGeom& g);
// ev0 / ev1 (optional) are recorded around the search kernel only.
hipError_t launch_dense(const DenseGeom& g, void* ws, float* ow, float* o1, int32_t* ok, hipStream_t s,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// One wave per pose: S_w and S_1 of arbitrary poses.
hipError_t launch_sparse(const void* field, int W, int H, int precision, const ModelPoint* pts, int n, int win,
                         const tm_eval_pose* poses, int np, float* scores, hipStream_t s);

// Candidate selection on a map (scratch: gw*gh entries of 32 bytes).
size_t select_workspace_bytes(int gw, int gh);
hipError_t launch_select(const float* sw, const float* s1, const int32_t* k, int gw, int gh, int sx, int sy,
                         int level, float min_score, double dmin2, double theta_min, double step_level,
                         tm_pose* out, int capacity, int32_t* n_out, void* scratch, hipStream_t s);

struct RefineLevel {
    const void* field;
    int W, H;
    const ModelPoint* pts;
    int n;
    double step;
    int K;
};

struct RefineArgs {
    RefineLevel lv[kMaxLevels];
    int L;                // levels present; poses above L-1 start at L-1
    int precision;
    int win;
    int full;             // wrap angle indices (else clamp)
    double theta_min;
};

// Refine poses[i] (i < *n_dev if n_dev, else i < n), all of level from_level,
// down to level 0, in place.  ws: refine_workspace_bytes(a, n) bytes.
size_t refine_workspace_bytes(const RefineArgs& a, int n);
hipError_t launch_refine(const RefineArgs& a, tm_pose* poses, int n, const int32_t* n_dev, int from_level, void* ws,
                         hipStream_t s);

// Final selection: S_w floor, key sort, greedy NMS at level 0, <= capacity.
hipError_t launch_final(const tm_pose* cand, const int32_t* n_cand, int max_cand, float min_score, double dmin2,
                        double theta_min, double step0, tm_pose* out, int capacity, int32_t* n_out, hipStream_t s);

}  // namespace tmk
