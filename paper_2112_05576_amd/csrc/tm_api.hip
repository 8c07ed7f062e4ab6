// C ABI of the template matcher: argument validation, handle and scratch
// management, and the order of kernel launches for each call.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <mutex>
#include <vector>

#include "tm_internal.h"

#define TM_EXPORT extern "C" __attribute__((visibility("default")))

namespace {

thread_local char g_err[512] = "";

tm_status fail(tm_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

tm_status hip_fail(hipError_t e, const char* where)
{
    return fail(e == hipErrorOutOfMemory ? TM_ENOMEM : TM_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

tm_status check_image(const uint8_t* img, int w, int h, int pitch, const tm_pyr_params* p, const char* what)
{
    if (!img) return fail(TM_EINVAL, "%s: null image", what);
    if (!p) return fail(TM_EINVAL, "%s: null params", what);
    if (p->levels < 1 || p->levels > TM_MAX_LEVELS)
        return fail(TM_EINVAL, "%s: levels must be in [1, %d], got %d", what, TM_MAX_LEVELS, p->levels);
    if (!(p->edge_thresh >= 0.0f) || !isfinite(p->edge_thresh))
        return fail(TM_EINVAL, "%s: edge_thresh must be finite and >= 0", what);
    if (p->precision != TM_FP32 && p->precision != TM_FP16)
        return fail(TM_EINVAL, "%s: precision must be TM_FP32 or TM_FP16", what);
    if (pitch < w) return fail(TM_EINVAL, "%s: pitch %d < width %d", what, pitch, w);
    const long long minside = 3LL << (p->levels - 1);
    if (w < minside || h < minside)
        return fail(TM_EINVAL, "%s: image %dx%d too small for %d levels (min side %lld)", what, w, h, p->levels,
                    minside);
    if ((long long)w * h > (1LL << 30)) return fail(TM_EINVAL, "%s: image too large", what);
    return TM_OK;
}

long long thresh_sq(float tau)
{
    double t2 = floor((double)tau * (double)tau);
    return t2 > 4e18 ? (long long)4e18 : (long long)t2;
}

void level_sizes(int w, int h, int L, int* ws, int* hs)
{
    ws[0] = w;
    hs[0] = h;
    for (int l = 1; l < L; ++l) {
        ws[l] = ws[l - 1] / 2;
        hs[l] = hs[l - 1] / 2;
    }
}

// ---------------------------------------------------------------- search grid
struct Grid {
    int L;
    double step[TM_MAX_LEVELS];
    int K[TM_MAX_LEVELS];
    int full;
};

tm_status check_search(const tm_search_params* sp, const char* what)
{
    if (!sp) return fail(TM_EINVAL, "%s: null search params", what);
    if (sp->step_x < 1 || sp->step_y < 1) return fail(TM_EINVAL, "%s: steps must be >= 1", what);
    if (!(sp->theta_step_top_deg > 0.0) || !isfinite(sp->theta_step_top_deg))
        return fail(TM_EINVAL, "%s: theta_step_top_deg must be > 0", what);
    if (!(sp->theta_range_deg > 0.0) || !isfinite(sp->theta_range_deg) || !isfinite(sp->theta_min_deg))
        return fail(TM_EINVAL, "%s: theta range must be finite and > 0", what);
    if (sp->neighbourhood < 1 || (sp->neighbourhood % 2) == 0 || sp->neighbourhood > 31)
        return fail(TM_EINVAL, "%s: neighbourhood must be odd in [1, 31]", what);
    if (sp->max_candidates < 1 || sp->max_candidates > 1024)
        return fail(TM_EINVAL, "%s: max_candidates must be in [1, 1024]", what);
    if (sp->max_matches < 1) return fail(TM_EINVAL, "%s: max_matches must be >= 1", what);
    if (!isfinite(sp->min_score) || !isfinite(sp->nms_min_dist))
        return fail(TM_EINVAL, "%s: min_score and nms_min_dist must be finite", what);
    return TM_OK;
}

tm_status make_grid(const tm_search_params* sp, int L, Grid* g)
{
    g->L = L;
    g->full = sp->theta_range_deg >= 360.0;
    for (int l = 0; l < L; ++l) {
        g->step[l] = ldexp(sp->theta_step_top_deg, -(L - 1 - l));
        double K = g->full ? ceil(360.0 / g->step[l]) : floor(sp->theta_range_deg / g->step[l] + 1e-9) + 1.0;
        if (K > 65535.0) return fail(TM_EINVAL, "angle grid too fine: %g angles at level %d", K, l);
        g->K[l] = (int)K;
    }
    return TM_OK;
}

// ---------------------------------------------------------------- timing
struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> used, free_;
};
Timing& timing()
{
    static Timing t;
    return t;
}

// An event pair to record around one search kernel, or (null, null) when
// timing is off.
tm_status timing_pair(hipEvent_t* a, hipEvent_t* b)
{
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    *a = *b = nullptr;
    if (!t.on) return TM_OK;
    std::pair<hipEvent_t, hipEvent_t> e;
    if (!t.free_.empty()) {
        e = t.free_.back();
        t.free_.pop_back();
    } else {
        HIP_TRY(hipEventCreate(&e.first));
        HIP_TRY(hipEventCreate(&e.second));
    }
    t.used.push_back(e);
    *a = e.first;
    *b = e.second;
    return TM_OK;
}

// ---------------------------------------------------------------- scratch
tm_status ensure_ws(tm_pyramid* p, size_t bytes, hipStream_t s)
{
    if (p->ws.bytes >= bytes) return TM_OK;
    if (p->ws.ptr) {
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipFree(p->ws.ptr));
        p->ws.ptr = nullptr;
        p->ws.bytes = 0;
    }
    bytes = align_up(bytes, 1 << 20);
    HIP_TRY(hipMalloc(&p->ws.ptr, bytes));
    p->ws.bytes = bytes;
    return TM_OK;
}

// Rotated table of the model's `level` for a grid; cached on the model.
tm_status get_table(const tm_model* mc, int level, double theta_min, double step, int K, hipStream_t s,
                    const tmk::TabEntry** out)
{
    tm_model* m = const_cast<tm_model*>(mc);
    tm_model_table_cache& c = m->cache;
    const tm_model_level& ml = m->lv[level];
    if (c.tab && c.level == level && c.theta_min == theta_min && c.step == step && c.K == K) {
        *out = c.tab;
        return TM_OK;
    }
    size_t need = (size_t)K * ml.n_pad;
    if (need > c.cap) {
        if (c.tab) {
            HIP_TRY(hipStreamSynchronize(s));
            HIP_TRY(hipFree(c.tab));
            c.tab = nullptr;
            c.cap = 0;
        }
        HIP_TRY(hipMalloc(&c.tab, need * sizeof(tmk::TabEntry)));
        c.cap = need;
    }
    HIP_TRY(tmk::launch_tables(ml.pts, ml.n, ml.n_pad, theta_min, step, K, c.tab, s));
    c.level = level;
    c.theta_min = theta_min;
    c.step = step;
    c.K = K;
    *out = c.tab;
    return TM_OK;
}

float default_dmin(const tm_model* m, const tm_search_params* sp)
{
    if (sp->nms_min_dist > 0.0f) return sp->nms_min_dist;
    return (float)(0.5 * sqrt((double)m->lv[0].radius2));
}

tm_status check_pair(const tm_model* m, const tm_pyramid* p, const char* what)
{
    if (!m || !p) return fail(TM_EINVAL, "%s: null model or pyramid", what);
    if (m->L < p->L)
        return fail(TM_EINVAL, "%s: model has %d levels, pyramid %d (model needs at least as many)", what, m->L,
                    p->L);
    return TM_OK;
}

tmk::RefineArgs refine_args(const tm_model* m, const tm_pyramid* p, const tm_search_params* sp, const Grid& g)
{
    tmk::RefineArgs a = {};
    for (int l = 0; l < p->L; ++l) {
        a.lv[l].field = p->lv[l].field;
        a.lv[l].W = p->lv[l].w;
        a.lv[l].H = p->lv[l].h;
        a.lv[l].pts = m->lv[l].pts;
        a.lv[l].n = m->lv[l].n;
        a.lv[l].step = g.step[l];
        a.lv[l].K = g.K[l];
    }
    a.L = p->L;
    a.precision = p->precision;
    a.win = sp->neighbourhood;
    a.full = g.full;
    a.theta_min = sp->theta_min_deg;
    return a;
}

tmk::DenseGeom dense_geom(const tm_model* m, const tm_pyramid* p, int level, const tm_search_params* sp,
                         const tmk::TabEntry* tab, int K)
{
    tmk::DenseGeom g;
    g.field = p->lv[level].field;
    g.W = p->lv[level].w;
    g.H = p->lv[level].h;
    g.precision = p->precision;
    g.tab = tab;
    g.n = m->lv[level].n;
    g.n_pad = m->lv[level].n_pad;
    g.K = K;
    g.sx = sp->step_x;
    g.sy = sp->step_y;
    g.win = sp->neighbourhood;
    g.rad = m->lv[level].rad;
    g.gw = (g.W + g.sx - 1) / g.sx;
    g.gh = (g.H + g.sy - 1) / g.sy;
    return g;
}

// scratch layout of detect: [dense partials][map w|1|k][select keys][cands][count][refine]
struct DetectLayout {
    size_t dense, map, sel, cand, refine, total;
};

DetectLayout detect_layout(const tmk::DenseGeom& g, int max_cand, size_t refine_bytes)
{
    DetectLayout d;
    const size_t np = (size_t)g.gw * g.gh;
    d.dense = 0;
    size_t off = align_up(tmk::dense_workspace_bytes(g), 256);
    d.map = off;
    off += align_up(np * 12, 256);
    d.sel = off;
    off += align_up(tmk::select_workspace_bytes(g.gw, g.gh), 256);
    d.cand = off;
    off += align_up((size_t)max_cand * sizeof(tm_pose) + 256, 256);
    d.refine = off;
    off += align_up(refine_bytes, 256);
    d.total = off;
    return d;
}

}  // namespace

// ======================================================================= API

TM_EXPORT const char* tm_last_error(void) { return g_err; }

TM_EXPORT const char* tm_version(void) { return "tm-hip 0.1 (gfx950)"; }

TM_EXPORT tm_status tm_build_pyramid(const uint8_t* img, int32_t w, int32_t h, int32_t pitch,
                                     const tm_pyr_params* pp, void* stream, tm_pyramid** out)
{
    g_err[0] = 0;
    if (!out) return fail(TM_EINVAL, "tm_build_pyramid: null out");
    *out = nullptr;
    tm_status st = check_image(img, w, h, pitch, pp, "tm_build_pyramid");
    if (st != TM_OK) return st;
    tm_pyramid* p = new (std::nothrow) tm_pyramid_s();
    if (!p) return fail(TM_ENOMEM, "tm_build_pyramid: host allocation");
    p->L = pp->levels;
    p->precision = pp->precision;
    p->tau = pp->edge_thresh;
    p->T2 = thresh_sq(pp->edge_thresh);
    hipGetDevice(&p->dev);
    int ws[TM_MAX_LEVELS], hs[TM_MAX_LEVELS];
    level_sizes(w, h, p->L, ws, hs);
    const size_t fsz = pp->precision == TM_FP16 ? 4 : 8;
    size_t total = 0;
    size_t img_off[TM_MAX_LEVELS], fld_off[TM_MAX_LEVELS];
    for (int l = 0; l < p->L; ++l) {
        img_off[l] = total;
        total = align_up(total + (size_t)ws[l] * hs[l], 256);
        fld_off[l] = total;
        total = align_up(total + (size_t)ws[l] * hs[l] * fsz, 256);
    }
    hipError_t e = hipMalloc(&p->block, total);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "tm_build_pyramid: hipMalloc");
    }
    for (int l = 0; l < p->L; ++l) {
        p->lv[l].w = ws[l];
        p->lv[l].h = hs[l];
        p->lv[l].img = reinterpret_cast<uint8_t*>(p->block) + img_off[l];
        p->lv[l].field = reinterpret_cast<uint8_t*>(p->block) + fld_off[l];
    }
    st = tm_update_pyramid(p, img, pitch, stream);
    if (st != TM_OK) {
        tm_pyramid_free(p);
        return st;
    }
    *out = p;
    return TM_OK;
}

TM_EXPORT tm_status tm_update_pyramid(tm_pyramid* p, const uint8_t* img, int32_t pitch, void* stream)
{
    if (!p || !img) return fail(TM_EINVAL, "tm_update_pyramid: null argument");
    if (pitch < p->lv[0].w) return fail(TM_EINVAL, "tm_update_pyramid: pitch %d < width %d", pitch, p->lv[0].w);
    HIP_TRY(tmk::launch_pyr_build(img, pitch, p->lv, p->L, S(stream)));
    HIP_TRY(tmk::launch_sobel_fields(p->lv, p->L, p->T2, p->precision, S(stream)));
    return TM_OK;
}

TM_EXPORT void tm_pyramid_free(tm_pyramid* p)
{
    if (!p) return;
    if (p->block) hipFree(p->block);
    if (p->ws.ptr) hipFree(p->ws.ptr);
    delete p;
}

TM_EXPORT tm_status tm_build_model(const uint8_t* img, int32_t w, int32_t h, int32_t pitch, const tm_pyr_params* pp,
                                   void* stream, tm_model** out)
{
    g_err[0] = 0;
    if (!out) return fail(TM_EINVAL, "tm_build_model: null out");
    *out = nullptr;
    tm_status st = check_image(img, w, h, pitch, pp, "tm_build_model");
    if (st != TM_OK) return st;
    hipStream_t s = S(stream);
    const int L = pp->levels;
    int ws[TM_MAX_LEVELS], hs[TM_MAX_LEVELS];
    level_sizes(w, h, L, ws, hs);
    // temporary uint8 pyramid and point buffers of full capacity
    tmk::PyrLevel lv[TM_MAX_LEVELS] = {};
    size_t total = 0, img_off[TM_MAX_LEVELS], pts_off[TM_MAX_LEVELS];
    for (int l = 0; l < L; ++l) {
        img_off[l] = total;
        total = align_up(total + (size_t)ws[l] * hs[l], 256);
    }
    for (int l = 0; l < L; ++l) {
        pts_off[l] = total;
        total = align_up(total + (size_t)ws[l] * hs[l] * sizeof(tmk::ModelPoint), 256);
    }
    const size_t cnt_off = total;
    total += 256;
    void* tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, total));
    tmk::ModelPoint* pts[TM_MAX_LEVELS];
    for (int l = 0; l < L; ++l) {
        lv[l].w = ws[l];
        lv[l].h = hs[l];
        lv[l].img = reinterpret_cast<uint8_t*>(tmp) + img_off[l];
        lv[l].field = nullptr;
        pts[l] = reinterpret_cast<tmk::ModelPoint*>(reinterpret_cast<uint8_t*>(tmp) + pts_off[l]);
    }
    int* counts = reinterpret_cast<int*>(reinterpret_cast<uint8_t*>(tmp) + cnt_off);
    const long long T2 = thresh_sq(pp->edge_thresh);
    hipError_t e = tmk::launch_pyr_build(img, pitch, lv, L, s);
    if (e == hipSuccess) e = tmk::launch_model_points(lv, L, T2, pts, counts, s);
    int hc[TM_MAX_LEVELS] = {};
    if (e == hipSuccess) e = hipMemcpyAsync(hc, counts, sizeof(int) * L, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        hipFree(tmp);
        return hip_fail(e, "tm_build_model");
    }
    for (int l = 0; l < L; ++l) {
        if (hc[l] < 1) {
            hipFree(tmp);
            return fail(TM_EINVAL, "tm_build_model: level %d has no edge point above the threshold", l);
        }
    }
    tm_model* m = new (std::nothrow) tm_model_s();
    if (!m) {
        hipFree(tmp);
        return fail(TM_ENOMEM, "tm_build_model: host allocation");
    }
    m->L = L;
    m->tau = pp->edge_thresh;
    hipGetDevice(&m->dev);
    for (int l = 0; l < L; ++l) {
        tm_model_level& ml = m->lv[l];
        ml.w = ws[l];
        ml.h = hs[l];
        ml.n = hc[l];
        ml.n_pad = (ml.n + 7) / 8 * 8;
        std::vector<tmk::ModelPoint> hp(ml.n);
        e = hipMemcpy(hp.data(), pts[l], sizeof(tmk::ModelPoint) * ml.n, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMalloc(&ml.pts, sizeof(tmk::ModelPoint) * ml.n);
        if (e == hipSuccess)
            e = hipMemcpy(ml.pts, hp.data(), sizeof(tmk::ModelPoint) * ml.n, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            hipFree(tmp);
            tm_model_free(m);
            return hip_fail(e, "tm_build_model: point copy");
        }
        int r2 = 0;
        for (const auto& q : hp) r2 = std::max(r2, (int)q.tx * q.tx + (int)q.ty * q.ty);
        ml.radius2 = r2;
        // |round(R t)| <= |t| + 1 per component
        ml.rad = (int)ceil(sqrt((double)r2)) + 1;
    }
    hipFree(tmp);
    *out = m;
    return TM_OK;
}

TM_EXPORT void tm_model_free(tm_model* m)
{
    if (!m) return;
    for (int l = 0; l < m->L; ++l)
        if (m->lv[l].pts) hipFree(m->lv[l].pts);
    if (m->cache.tab) hipFree(m->cache.tab);
    delete m;
}

TM_EXPORT tm_status tm_model_level_info(const tm_model* m, int32_t level, int32_t* w, int32_t* h, int32_t* n)
{
    if (!m) return fail(TM_EINVAL, "tm_model_level_info: null model");
    if (level < 0 || level >= m->L) return fail(TM_EINVAL, "tm_model_level_info: bad level %d", level);
    if (w) *w = m->lv[level].w;
    if (h) *h = m->lv[level].h;
    if (n) *n = m->lv[level].n;
    return TM_OK;
}

namespace {
__global__ void k_points_export(const tmk::ModelPoint* __restrict__ p, int n, int32_t* __restrict__ t,
                                int32_t* __restrict__ g)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tmk::ModelPoint q = p[i];
    if (t) {
        t[2 * i] = q.tx;
        t[2 * i + 1] = q.ty;
    }
    if (g) {
        g[2 * i] = q.gx;
        g[2 * i + 1] = q.gy;
    }
}
}  // namespace

TM_EXPORT tm_status tm_model_points(const tm_model* m, int32_t level, int32_t* t, int32_t* g, void* stream)
{
    if (!m) return fail(TM_EINVAL, "tm_model_points: null model");
    if (level < 0 || level >= m->L) return fail(TM_EINVAL, "tm_model_points: bad level %d", level);
    const int n = m->lv[level].n;
    hipLaunchKernelGGL(k_points_export, dim3((n + 255) / 256), dim3(256), 0, S(stream), m->lv[level].pts, n, t, g);
    HIP_TRY(hipGetLastError());
    return TM_OK;
}

TM_EXPORT tm_status tm_model_table(const tm_model* m, int32_t level, double theta_min, double step, int32_t K,
                                   int32_t* q, float* r, void* stream)
{
    if (!m || !q || !r) return fail(TM_EINVAL, "tm_model_table: null argument");
    if (level < 0 || level >= m->L) return fail(TM_EINVAL, "tm_model_table: bad level %d", level);
    if (K < 1 || K > 65535 || !(step > 0.0)) return fail(TM_EINVAL, "tm_model_table: bad angle grid");
    const tmk::TabEntry* tab = nullptr;
    tm_status st = get_table(m, level, theta_min, step, K, S(stream), &tab);
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_table_export(tab, m->lv[level].n, m->lv[level].n_pad, K, q, r, S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_pyramid_level(const tm_pyramid* p, int32_t level, int32_t* w, int32_t* h,
                                     const uint8_t** img, const void** field, int32_t* precision)
{
    if (!p) return fail(TM_EINVAL, "tm_pyramid_level: null pyramid");
    if (level < 0 || level >= p->L) return fail(TM_EINVAL, "tm_pyramid_level: bad level %d", level);
    if (w) *w = p->lv[level].w;
    if (h) *h = p->lv[level].h;
    if (img) *img = p->lv[level].img;
    if (field) *field = p->lv[level].field;
    if (precision) *precision = p->precision;
    return TM_OK;
}

TM_EXPORT tm_status tm_pyramid_read(const tm_pyramid* p, int32_t level, uint8_t* img, void* field, void* stream)
{
    if (!p) return fail(TM_EINVAL, "tm_pyramid_read: null pyramid");
    if (level < 0 || level >= p->L) return fail(TM_EINVAL, "tm_pyramid_read: bad level %d", level);
    const size_t np = (size_t)p->lv[level].w * p->lv[level].h;
    if (img) HIP_TRY(hipMemcpyAsync(img, p->lv[level].img, np, hipMemcpyDeviceToDevice, S(stream)));
    if (field)
        HIP_TRY(hipMemcpyAsync(field, p->lv[level].field, np * (p->precision == TM_FP16 ? 4 : 8),
                               hipMemcpyDeviceToDevice, S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_score_poses(const tm_model* m, const tm_pyramid* p, int32_t level, int32_t win,
                                   const tm_eval_pose* poses, int32_t n, float* scores, void* stream)
{
    tm_status st = check_pair(m, p, "tm_score_poses");
    if (st != TM_OK) return st;
    if (level < 0 || level >= p->L) return fail(TM_EINVAL, "tm_score_poses: bad level %d", level);
    if (win < 1 || win % 2 == 0 || win > 31) return fail(TM_EINVAL, "tm_score_poses: window must be odd in [1, 31]");
    if (n < 0) return fail(TM_EINVAL, "tm_score_poses: n < 0");
    if (n > 0 && (!poses || !scores)) return fail(TM_EINVAL, "tm_score_poses: null buffer");
    HIP_TRY(tmk::launch_sparse(p->lv[level].field, p->lv[level].w, p->lv[level].h, p->precision, m->lv[level].pts,
                              m->lv[level].n, win, poses, n, scores, S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_score_map(const tm_model* m, tm_pyramid* p, int32_t level, const tm_search_params* sp,
                                 float* sw, float* s1, int32_t* k, void* stream)
{
    tm_status st = check_pair(m, p, "tm_score_map");
    if (st != TM_OK) return st;
    st = check_search(sp, "tm_score_map");
    if (st != TM_OK) return st;
    if (level < 0 || level >= p->L) return fail(TM_EINVAL, "tm_score_map: bad level %d", level);
    if (!sw || !s1 || !k) return fail(TM_EINVAL, "tm_score_map: null output");
    Grid g;
    st = make_grid(sp, p->L, &g);
    if (st != TM_OK) return st;
    hipStream_t s = S(stream);
    const tmk::TabEntry* tab = nullptr;
    st = get_table(m, level, sp->theta_min_deg, g.step[level], g.K[level], s, &tab);
    if (st != TM_OK) return st;
    tmk::DenseGeom dg = dense_geom(m, p, level, sp, tab, g.K[level]);
    st = ensure_ws(p, tmk::dense_workspace_bytes(dg), s);
    if (st != TM_OK) return st;
    hipEvent_t ev0, ev1;
    st = timing_pair(&ev0, &ev1);
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_dense(dg, p->ws.ptr, sw, s1, k, s, ev0, ev1));
    return TM_OK;
}

TM_EXPORT tm_status tm_select(const float* sw, const float* s1, const int32_t* k, int32_t gw, int32_t gh,
                              int32_t sx, int32_t sy, int32_t level, float min_score, float dmin, tm_pose* out,
                              int32_t capacity, int32_t* n_out, void* stream)
{
    if (!sw || !s1 || !k || !out || !n_out) return fail(TM_EINVAL, "tm_select: null argument");
    if (gw < 1 || gh < 1 || sx < 1 || sy < 1 || level < 0 || level >= 31)
        return fail(TM_EINVAL, "tm_select: bad geometry");
    if (capacity < 1 || capacity > 1024) return fail(TM_EINVAL, "tm_select: capacity must be in [1, 1024]");
    if (!isfinite(min_score) || !isfinite(dmin)) return fail(TM_EINVAL, "tm_select: non-finite threshold");
    // scratch comes from a small private buffer (this entry point has no pyramid)
    static thread_local void* scratch = nullptr;
    static thread_local size_t scratch_bytes = 0;
    size_t need = tmk::select_workspace_bytes(gw, gh);
    hipStream_t s = S(stream);
    if (need > scratch_bytes) {
        if (scratch) {
            HIP_TRY(hipStreamSynchronize(s));
            HIP_TRY(hipFree(scratch));
            scratch = nullptr;
            scratch_bytes = 0;
        }
        HIP_TRY(hipMalloc(&scratch, need));
        scratch_bytes = need;
    }
    const double dmin2 = (double)dmin * (double)dmin;
    HIP_TRY(tmk::launch_select(sw, s1, k, gw, gh, sx, sy, level, min_score, dmin2, 0.0, 0.0, out, capacity, n_out,
                              scratch, s));
    return TM_OK;
}

TM_EXPORT tm_status tm_detect(const tm_model* m, tm_pyramid* p, const tm_search_params* sp, tm_pose* out,
                              int32_t capacity, int32_t* n_out, void* stream)
{
    tm_status st = check_pair(m, p, "tm_detect");
    if (st != TM_OK) return st;
    st = check_search(sp, "tm_detect");
    if (st != TM_OK) return st;
    if (!out || !n_out) return fail(TM_EINVAL, "tm_detect: null output");
    if (capacity < 1) return fail(TM_EINVAL, "tm_detect: capacity < 1");
    Grid g;
    st = make_grid(sp, p->L, &g);
    if (st != TM_OK) return st;
    hipStream_t s = S(stream);
    const int top = p->L - 1;
    const tmk::TabEntry* tab = nullptr;
    st = get_table(m, top, sp->theta_min_deg, g.step[top], g.K[top], s, &tab);
    if (st != TM_OK) return st;
    tmk::DenseGeom dg = dense_geom(m, p, top, sp, tab, g.K[top]);
    tmk::RefineArgs ra = refine_args(m, p, sp, g);
    DetectLayout lay = detect_layout(dg, sp->max_candidates, tmk::refine_workspace_bytes(ra, sp->max_candidates));
    st = ensure_ws(p, lay.total, s);
    if (st != TM_OK) return st;
    uint8_t* base = reinterpret_cast<uint8_t*>(p->ws.ptr);
    const size_t np = (size_t)dg.gw * dg.gh;
    float* mw = reinterpret_cast<float*>(base + lay.map);
    float* m1 = mw + np;
    int32_t* mk = reinterpret_cast<int32_t*>(m1 + np);
    tm_pose* cand = reinterpret_cast<tm_pose*>(base + lay.cand);
    int32_t* ncand = reinterpret_cast<int32_t*>(base + lay.cand + (size_t)sp->max_candidates * sizeof(tm_pose));
    const float dmin = default_dmin(m, sp);
    const double dmin2 = (double)dmin * (double)dmin;
    hipEvent_t ev0, ev1;
    st = timing_pair(&ev0, &ev1);
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_dense(dg, base + lay.dense, mw, m1, mk, s, ev0, ev1));
    HIP_TRY(tmk::launch_select(mw, m1, mk, dg.gw, dg.gh, sp->step_x, sp->step_y, top, sp->min_score, dmin2,
                              sp->theta_min_deg, g.step[top], cand, sp->max_candidates, ncand, base + lay.sel, s));
    if (p->L > 1) HIP_TRY(tmk::launch_refine(ra, cand, sp->max_candidates, ncand, top, base + lay.refine, s));
    const int cap = std::min(capacity, sp->max_matches);
    HIP_TRY(tmk::launch_final(cand, ncand, sp->max_candidates, sp->min_score, dmin2, sp->theta_min_deg, g.step[0],
                             out, cap, n_out, s));
    return TM_OK;
}

TM_EXPORT tm_status tm_timing_enable(int32_t on)
{
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    t.on = on != 0;
    return TM_OK;
}

TM_EXPORT tm_status tm_timing_read(double* ms, int32_t* launches)
{
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    double total = 0.0;
    for (auto& e : t.used) {
        HIP_TRY(hipEventSynchronize(e.second));
        float v = 0.f;
        HIP_TRY(hipEventElapsedTime(&v, e.first, e.second));
        total += v;
    }
    if (ms) *ms = total;
    if (launches) *launches = (int32_t)t.used.size();
    t.free_.insert(t.free_.end(), t.used.begin(), t.used.end());
    t.used.clear();
    return TM_OK;
}

TM_EXPORT tm_status tm_refine(const tm_model* m, tm_pyramid* p, const tm_search_params* sp, int32_t from_level,
                              tm_pose* poses, int32_t n, void* stream)
{
    tm_status st = check_pair(m, p, "tm_refine");
    if (st != TM_OK) return st;
    st = check_search(sp, "tm_refine");
    if (st != TM_OK) return st;
    if (n < 0) return fail(TM_EINVAL, "tm_refine: n < 0");
    if (n == 0) return TM_OK;
    if (!poses) return fail(TM_EINVAL, "tm_refine: null poses");
    Grid g;
    st = make_grid(sp, p->L, &g);
    if (st != TM_OK) return st;
    if (from_level < 0 || from_level >= p->L) return fail(TM_EINVAL, "tm_refine: bad from_level %d", from_level);
    tmk::RefineArgs ra = refine_args(m, p, sp, g);
    st = ensure_ws(p, tmk::refine_workspace_bytes(ra, n), S(stream));
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_refine(ra, poses, n, nullptr, from_level, p->ws.ptr, S(stream)));
    return TM_OK;
}
