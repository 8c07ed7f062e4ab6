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

// ---------------------------------------------------------------- allocator
// The allocator new handles take (tm_set_allocator); each handle keeps a copy.
std::mutex g_alloc_mu;
tm_allocator g_alloc = {nullptr, nullptr, nullptr};

tm_allocator current_allocator()
{
    std::lock_guard<std::mutex> g(g_alloc_mu);
    return g_alloc;
}

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
    if (p->source != TM_PYR_GREY && p->source != TM_PYR_GRADIENT)
        return fail(TM_EINVAL, "%s: source must be TM_PYR_GREY or TM_PYR_GRADIENT", what);
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
    int S;                         // scales
    double sigma_min, sigma_step;  // scale grid
    double sigma_max;              // largest scale (>= 1 for the radius bounds)
};

// Bound on |q| components of a model level's points over all angles at
// scales up to sigma_max: |round(sigma R t)| <= sigma |t| + 1.
int scaled_rad(const tm_model_level& ml, double sigma_max)
{
    if (sigma_max <= 1.0) return ml.rad;
    return std::max(ml.rad, (int)ceil(sigma_max * sqrt((double)ml.radius2)) + 1);
}

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
    if (sp->scale_count < 1 || sp->scale_count > 64) return fail(TM_EINVAL, "%s: scale_count must be 1..64", what);
    if (!(sp->scale_min > 0.0) || !isfinite(sp->scale_min) || !(sp->scale_step >= 0.0) || !isfinite(sp->scale_step))
        return fail(TM_EINVAL, "%s: scale_min must be > 0 and scale_step >= 0", what);
    if (sp->scale_min + (sp->scale_count - 1) * sp->scale_step > 16.0)
        return fail(TM_EINVAL, "%s: scales above 16", what);
    if (sp->vote != TM_VOTE_ALL && sp->vote != TM_VOTE_EDGE)
        return fail(TM_EINVAL, "%s: vote must be TM_VOTE_ALL or TM_VOTE_EDGE", what);
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
    g->S = sp->scale_count;
    g->sigma_min = sp->scale_min;
    g->sigma_step = sp->scale_step;
    g->sigma_max = std::max(1.0, sp->scale_min + (sp->scale_count - 1) * sp->scale_step);
    if ((long long)g->K[L - 1] * g->S > 65535)
        return fail(TM_EINVAL, "%d angles x %d scales at the top level: more than 65535 poses per translation",
                    g->K[L - 1], g->S);
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
        tmk::dev_free(p->alloc, p->ws.ptr, s);
        p->ws.ptr = nullptr;
        p->ws.bytes = 0;
    }
    bytes = align_up(bytes, 1 << 20);
    HIP_TRY(tmk::dev_alloc(p->alloc, &p->ws.ptr, bytes, s));
    p->ws.bytes = bytes;
    p->desc_valid = false;
    return TM_OK;
}

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Rotated table of the model's `level` for a grid, cached on the model per
// (level, grid): a new grid gets a table of its own (built on stream s, an
// event recorded after it) and earlier tables stay valid for the streams
// still reading them.  A stream other than the builder's waits for the event.
constexpr size_t kMaxTables = 32;  // tables cached per model

tm_status get_table(const tm_model* mc, int level, double theta_min, double step, int K, const Grid& g,
                    hipStream_t s, const tmk::TabEntry** out)
{
    tm_model* m = const_cast<tm_model*>(mc);
    const tm_model_level& ml = m->lv[level];
    if (scaled_rad(ml, g.sigma_max) > 32000) return fail(TM_EINVAL, "model too large for the scale range");
    std::lock_guard<std::mutex> lock(m->mu);
    for (const tm_rot_table& c : m->tables) {
        if (c.level == level && c.theta_min == theta_min && c.step == step && c.K == K && c.S == g.S &&
            c.sigma_min == g.sigma_min && c.sigma_step == g.sigma_step) {
            if (c.stream != s) {
                if (!stream_capturing(s)) {
                    HIP_TRY(hipStreamWaitEvent(s, c.ready, 0));
                } else if (hipEventQuery(c.ready) != hipSuccess) {
                    return fail(TM_EINVAL, "rotated table still being built on another stream; wait for it before "
                                           "capturing");
                }
            }
            *out = c.tab;
            return TM_OK;
        }
    }
    if (stream_capturing(s))
        return fail(TM_EINVAL, "no rotated table for this grid yet; run the call once before capturing");
    if (m->tables.size() >= kMaxTables) {
        // evict the oldest table once the device has passed every use of it
        HIP_TRY(hipDeviceSynchronize());
        tm_rot_table& o = m->tables.front();
        tmk::dev_free(m->alloc, o.tab, s);
        (void)hipEventDestroy(o.ready);
        m->tables.erase(m->tables.begin());
    }
    tm_rot_table c;
    c.level = level;
    c.theta_min = theta_min;
    c.step = step;
    c.K = K;
    c.S = g.S;
    c.sigma_min = g.sigma_min;
    c.sigma_step = g.sigma_step;
    c.stream = s;
    void* tab = nullptr;
    HIP_TRY(tmk::dev_alloc(m->alloc, &tab, (size_t)K * g.S * ml.n_pad * sizeof(tmk::TabEntry), s));
    c.tab = reinterpret_cast<tmk::TabEntry*>(tab);
    hipError_t e = hipEventCreateWithFlags(&c.ready, hipEventDisableTiming);
    if (e == hipSuccess)
        e = tmk::launch_tables(ml.pts, ml.n, ml.n_pad, theta_min, step, K, g.sigma_min, g.sigma_step, g.S, c.tab, s);
    if (e == hipSuccess) e = hipEventRecord(c.ready, s);
    if (e != hipSuccess) {
        if (c.ready) (void)hipEventDestroy(c.ready);
        tmk::dev_free(m->alloc, tab, s);
        return hip_fail(e, "rotated table");
    }
    m->tables.push_back(c);
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

tmk::SearchDesc make_search(const tm_search_params* sp, const Grid& g, int level, int precision, int capacity)
{
    tmk::SearchDesc s;
    memset(&s, 0, sizeof(s));
    s.L = g.L;
    s.level = level;
    for (int l = 0; l < g.L; ++l) {
        s.K[l] = g.K[l];
        s.step[l] = g.step[l];
    }
    s.theta_min = sp->theta_min_deg;
    s.full = g.full;
    s.win = sp->neighbourhood;
    s.vote = sp->vote;
    s.sx = sp->step_x;
    s.sy = sp->step_y;
    s.precision = precision;
    s.min_score = sp->min_score;
    s.max_cand = sp->max_candidates;
    s.capacity = capacity;
    s.max_matches = sp->max_matches;
    s.S = g.S;
    s.sigma_min = g.sigma_min;
    s.sigma_step = g.sigma_step;
    return s;
}

tmk::PairGeom pair_geom(const tm_model* m, const tm_pyramid* p, int level, int sx, int sy, double sigma_max)
{
    tmk::PairGeom g;
    g.W = p->lv[level].w;
    g.H = p->lv[level].h;
    g.gw = (g.W + sx - 1) / sx;
    g.gh = (g.H + sy - 1) / sy;
    g.rad = scaled_rad(m->lv[level], sigma_max);
    g.n = m->lv[level].n;
    return g;
}

// Static part of a pair descriptor: the image's levels, the model's levels,
// the rotated table of the searched level and the suppression distance.
void pair_static(tmk::PairDesc* d, const tm_model* m, const tm_pyramid* p, const tmk::TabEntry* tab, int level,
                 const tmk::PairGeom& g, const tmk::DensePlan& plan, float dmin, int win, double sigma_max)
{
    for (int l = 0; l < p->L; ++l) {
        d->field[l] = p->lv[l].field32;  // the refinement and the re-scoring work in FP32
        d->W[l] = p->lv[l].w;
        d->H[l] = p->lv[l].h;
        d->pts[l] = m->lv[l].pts;
        d->dir[l] = m->lv[l].dir;
        d->n[l] = m->lv[l].n;
        d->rad_l[l] = scaled_rad(m->lv[l], sigma_max);
        d->rtile[l] = tmk::refine_tile_fits(d->rad_l[l], TM_FP32, win) ? 1 : 0;
    }
    d->sfield = p->lv[level].field;  // the exhaustive search reads the storage precision
    d->tab = tab;
    d->n_pad = m->lv[level].n_pad;
    d->rad = g.rad;
    d->gw = g.gw;
    d->gh = g.gh;
    tmk::plan_tiles(plan, g, &d->tiles_x, &d->tiles_y);
    d->dmin = dmin;
}

// Scratch of one pair placed at `base` (null: measure only); returns bytes.
// search: chunk partials and the best-angle map; select: selection scratch
// and the candidate list; refine: centres and partial sums per level.
size_t pair_scratch(tmk::PairDesc* d, const tm_model* m, const tmk::PairGeom& g, const tmk::DensePlan& plan, int L,
                    int max_cand, bool search, bool select, bool refine, uint8_t* base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> uint8_t* {
        uint8_t* r = base ? base + off : nullptr;
        off = align_up(off + bytes, 256);
        return r;
    };
    const size_t np = (size_t)g.gw * g.gh;
    if (search) {
        const size_t C = (size_t)plan.C;
        float* pw = reinterpret_cast<float*>(take(tmk::dense_partials_bytes(plan, (int)np)));
        float* mw = reinterpret_cast<float*>(take(np * (plan.screen ? 24 : 12)));
        if (!plan.fast) {
            // the generic search's zero-bordered copy of the searched field
            const int pad = g.rad + plan.win_h + 1;
            const int pW = g.W + 2 * pad, pH = g.H + 2 * pad;
            uint8_t* pf = take((size_t)pW * pH * plan.px_bytes);
            if (base) {
                d->pfield = pf;
                d->pW = pW;
                d->pH = pH;
                d->pad = pad;
            }
        }
        if (base) {
            d->pw = pw;
            d->p1 = pw + C * np;
            d->pk = reinterpret_cast<int32_t*>(pw + 2 * C * np);
            d->mw = mw;
            d->m1 = mw + np;
            d->mk = reinterpret_cast<int32_t*>(mw + 2 * np);
            if (plan.screen) {
                d->p2 = pw + 3 * C * np;
                d->pk2 = reinterpret_cast<int32_t*>(pw + 4 * C * np);
                d->p3 = pw + 5 * C * np;
                d->m2 = mw + 3 * np;
                d->mk2 = reinterpret_cast<int32_t*>(mw + 4 * np);
                d->m3 = mw + 5 * np;
            }
        }
    }
    if (select) {
        float* sel = reinterpret_cast<float*>(take(tmk::select_scratch_bytes((int)np)));
        uint8_t* cp = take((size_t)max_cand * sizeof(tm_pose) + 256);
        if (base) {
            d->sel = sel;
            d->cand = reinterpret_cast<tm_pose*>(cp);
            d->ncand = reinterpret_cast<int32_t*>(cp + (size_t)max_cand * sizeof(tm_pose));
        }
    }
    if (refine) {
        tm_pose* c0 = reinterpret_cast<tm_pose*>(take((size_t)max_cand * sizeof(tm_pose)));
        tm_pose* c1 = reinterpret_cast<tm_pose*>(take((size_t)max_cand * sizeof(tm_pose)));
        if (base) {
            d->ctr[0] = c0;
            d->ctr[1] = c1;
        }
        for (int l = 0; l < L; ++l) {
            float* pl = reinterpret_cast<float*>(
                take((size_t)max_cand * tmk::kPartPerCand * sizeof(float)));
            if (base) d->part[l] = pl;
        }
    }
    return off;
}

__global__ void k_put_desc(tmk::PairDesc d, tmk::PairDesc* dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = d;
}

constexpr size_t kDescBytes = 4096;  // reserved at the start of a pyramid's scratch for its descriptor
static_assert(sizeof(tmk::PairDesc) <= 1024, "descriptor cache");

// Device copy of a one-pair descriptor at the start of the pyramid's scratch,
// enqueued only when it differs from the last one written there.
tm_status put_desc(tm_pyramid* p, const tmk::PairDesc& d, hipStream_t s, tmk::PairDesc** out)
{
    tmk::PairDesc* dev = reinterpret_cast<tmk::PairDesc*>(p->ws.ptr);
    if (!p->desc_valid || memcmp(p->last_desc, &d, sizeof(d)) != 0) {
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, dev);
        HIP_TRY(hipGetLastError());
        memcpy(p->last_desc, &d, sizeof(d));
        p->desc_valid = true;
    }
    *out = dev;
    return TM_OK;
}

// Per level: the pairs refined by gathers and by the staged kernel (the same
// rule as pair_static), with the grid and LDS sizes of each launch.  Staging
// is used once a launch refines at least kStagedMin candidates.
constexpr int kStagedMin = 512;

tmk::RefinePlan refine_plan(const tm_model* const* models, int n_models, int L, int win, long long candidates,
                            double sigma_max)
{
    const int precision = TM_FP32;  // the refinement reads the FP32 fields (an FP16 pyramid's twin)
    tmk::RefinePlan rp;
    memset(&rp, 0, sizeof(rp));
    rp.staged = candidates >= kStagedMin;
    for (int l = 0; l < L; ++l)
        for (int j = 0; j < n_models; ++j) {
            const int rad = scaled_rad(models[j]->lv[l], sigma_max);
            if (tmk::refine_tile_fits(rad, precision, win))
                rp.tile_bytes[l] = std::max(rp.tile_bytes[l], (int)tmk::refine_tile_bytes(rad, precision));
            else
                rp.gather[l] = 1;
        }
    return rp;
}

}  // namespace

// ======================================================================= API

TM_EXPORT const char* tm_last_error(void) { return g_err; }

namespace tmk {
hipError_t dev_alloc(const tm_allocator& a, void** p, size_t bytes, hipStream_t s)
{
    *p = nullptr;
    if (!a.alloc) return hipMalloc(p, bytes);
    void* q = a.alloc(bytes, a.ctx, reinterpret_cast<void*>(s));
    if (!q) return hipErrorOutOfMemory;
    if ((reinterpret_cast<uintptr_t>(q) & 255u) != 0) {  // the layouts assume 256-byte alignment
        a.free(q, a.ctx, reinterpret_cast<void*>(s));
        return hipErrorInvalidValue;
    }
    *p = q;
    return hipSuccess;
}

void dev_free(const tm_allocator& a, void* p, hipStream_t s)
{
    if (!p) return;
    if (a.free)
        a.free(p, a.ctx, reinterpret_cast<void*>(s));
    else
        (void)hipFree(p);
}
}  // namespace tmk

TM_EXPORT tm_status tm_set_allocator(const tm_allocator* a)
{
    if (a && ((a->alloc == nullptr) != (a->free == nullptr)))
        return fail(TM_EINVAL, "tm_set_allocator: give both alloc and free, or neither");
    std::lock_guard<std::mutex> g(g_alloc_mu);
    if (a && a->alloc)
        g_alloc = *a;
    else
        g_alloc = tm_allocator{nullptr, nullptr, nullptr};
    return TM_OK;
}

TM_EXPORT const char* tm_version(void) { return "tm-hip 0.1 (gfx950)"; }

namespace {
// A pyramid of a w x h image with storage for all levels (not yet built).
// top_only_fp16: an FP16 pyramid of a batch, whose levels below the top are
// only ever read in FP32 (by the refinement): their FP16 field is neither
// allocated nor written (lv[l].field is null there).
tm_status alloc_pyramid(int w, int h, const tm_pyr_params* pp, hipStream_t s, tm_pyramid** out,
                        bool top_only_fp16 = false)
{
    tm_pyramid* p = new (std::nothrow) tm_pyramid_s();
    if (!p) return fail(TM_ENOMEM, "pyramid: host allocation");
    p->alloc = current_allocator();
    p->L = pp->levels;
    p->precision = pp->precision;
    p->source = pp->source;
    p->tau = pp->edge_thresh;
    p->T2 = thresh_sq(pp->edge_thresh);
    if (hipGetDevice(&p->dev) != hipSuccess) {
        delete p;
        return fail(TM_EDEVICE, "pyramid: hipGetDevice");
    }
    int ws[TM_MAX_LEVELS], hs[TM_MAX_LEVELS];
    level_sizes(w, h, p->L, ws, hs);
    // per level: the uint8 image, the direction field in the storage
    // precision, for FP16 its FP32 twin, and the gradient maps if asked for
    const bool fp16 = pp->precision == TM_FP16;
    const size_t fsz = fp16 ? 4 : 8;
    size_t total = 0;
    size_t img_off[TM_MAX_LEVELS], fld_off[TM_MAX_LEVELS], f32_off[TM_MAX_LEVELS], grd_off[TM_MAX_LEVELS];
    const bool gradient = pp->source == TM_PYR_GRADIENT;
    bool has_field[TM_MAX_LEVELS];
    for (int l = 0; l < p->L; ++l) {
        img_off[l] = total;
        total = align_up(total + (size_t)ws[l] * hs[l], 256);
        fld_off[l] = total;
        has_field[l] = !(fp16 && top_only_fp16 && l < p->L - 1);
        if (has_field[l]) total = align_up(total + (size_t)ws[l] * hs[l] * fsz, 256);
        f32_off[l] = fp16 ? total : fld_off[l];
        if (fp16) total = align_up(total + (size_t)ws[l] * hs[l] * 8, 256);
        grd_off[l] = total;
        if (gradient) total = align_up(total + (size_t)ws[l] * hs[l] * 4, 256);
    }
    hipError_t e = tmk::dev_alloc(p->alloc, &p->block, total, s);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "pyramid: device allocation");
    }
    for (int l = 0; l < p->L; ++l) {
        p->lv[l].w = ws[l];
        p->lv[l].h = hs[l];
        p->lv[l].img = reinterpret_cast<uint8_t*>(p->block) + img_off[l];
        p->lv[l].field = has_field[l] ? reinterpret_cast<uint8_t*>(p->block) + fld_off[l] : nullptr;
        p->lv[l].field32 = reinterpret_cast<uint8_t*>(p->block) + f32_off[l];
        p->lv[l].grad = gradient ? reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(p->block) + grd_off[l])
                                 : nullptr;
    }
    *out = p;
    return TM_OK;
}
}  // namespace

TM_EXPORT tm_status tm_build_pyramid(const uint8_t* img, int32_t w, int32_t h, int32_t pitch,
                                     const tm_pyr_params* pp, void* stream, tm_pyramid** out)
{
    g_err[0] = 0;
    if (!out) return fail(TM_EINVAL, "tm_build_pyramid: null out");
    *out = nullptr;
    tm_status st = check_image(img, w, h, pitch, pp, "tm_build_pyramid");
    if (st != TM_OK) return st;
    tm_pyramid* p = nullptr;
    st = alloc_pyramid(w, h, pp, S(stream), &p);
    if (st != TM_OK) return st;
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
    if (p->source == TM_PYR_GRADIENT) HIP_TRY(tmk::launch_grad_pyramid(p->lv, p->L, S(stream)));
    HIP_TRY(tmk::launch_sobel_fields(p->lv, p->L, p->T2, p->precision, S(stream)));
    return TM_OK;
}

TM_EXPORT void tm_pyramid_free(tm_pyramid* p)
{
    if (!p) return;
    tmk::dev_free(p->alloc, p->block, nullptr);
    tmk::dev_free(p->alloc, p->ws.ptr, nullptr);
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
    size_t total = 0, img_off[TM_MAX_LEVELS], pts_off[TM_MAX_LEVELS], grd_off[TM_MAX_LEVELS];
    const bool gradient = pp->source == TM_PYR_GRADIENT;
    for (int l = 0; l < L; ++l) {
        img_off[l] = total;
        total = align_up(total + (size_t)ws[l] * hs[l], 256);
        grd_off[l] = total;
        if (gradient) total = align_up(total + (size_t)ws[l] * hs[l] * 4, 256);
    }
    for (int l = 0; l < L; ++l) {
        pts_off[l] = total;
        total = align_up(total + (size_t)ws[l] * hs[l] * sizeof(tmk::ModelPoint), 256);
    }
    const size_t cnt_off = total;
    total += 256;
    const tm_allocator A = current_allocator();
    void* tmp = nullptr;
    HIP_TRY(tmk::dev_alloc(A, &tmp, total, s));
    tmk::ModelPoint* pts[TM_MAX_LEVELS];
    for (int l = 0; l < L; ++l) {
        lv[l].w = ws[l];
        lv[l].h = hs[l];
        lv[l].img = reinterpret_cast<uint8_t*>(tmp) + img_off[l];
        lv[l].field = nullptr;
        lv[l].grad = gradient ? reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(tmp) + grd_off[l]) : nullptr;
        pts[l] = reinterpret_cast<tmk::ModelPoint*>(reinterpret_cast<uint8_t*>(tmp) + pts_off[l]);
    }
    int* counts = reinterpret_cast<int*>(reinterpret_cast<uint8_t*>(tmp) + cnt_off);
    const long long T2 = thresh_sq(pp->edge_thresh);
    hipError_t e = tmk::launch_pyr_build(img, pitch, lv, L, s);
    if (e == hipSuccess && gradient) e = tmk::launch_grad_pyramid(lv, L, s);
    if (e == hipSuccess) e = tmk::launch_model_points(lv, L, T2, pts, counts, s);
    int hc[TM_MAX_LEVELS] = {};
    if (e == hipSuccess) e = hipMemcpyAsync(hc, counts, sizeof(int) * L, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        tmk::dev_free(A, tmp, s);
        return hip_fail(e, "tm_build_model");
    }
    for (int l = 0; l < L; ++l) {
        if (hc[l] < 1) {
            tmk::dev_free(A, tmp, s);
            return fail(TM_EINVAL, "tm_build_model: level %d has no edge point above the threshold", l);
        }
    }
    tm_model* m = new (std::nothrow) tm_model_s();
    if (!m) {
        tmk::dev_free(A, tmp, s);
        return fail(TM_ENOMEM, "tm_build_model: host allocation");
    }
    m->alloc = A;
    m->L = L;
    m->tau = pp->edge_thresh;
    m->source = pp->source;
    if (hipGetDevice(&m->dev) != hipSuccess) {
        tmk::dev_free(A, tmp, s);
        delete m;
        return fail(TM_EDEVICE, "tm_build_model: hipGetDevice");
    }
    for (int l = 0; l < L; ++l) {
        tm_model_level& ml = m->lv[l];
        ml.w = ws[l];
        ml.h = hs[l];
        ml.n = hc[l];
        ml.n_pad = (ml.n + 7) / 8 * 8;
        std::vector<tmk::ModelPoint> hp(ml.n);
        e = hipMemcpy(hp.data(), pts[l], sizeof(tmk::ModelPoint) * ml.n, hipMemcpyDeviceToHost);
        void* vp = nullptr;
        if (e == hipSuccess) e = tmk::dev_alloc(A, &vp, sizeof(tmk::ModelPoint) * ml.n, s);
        ml.pts = reinterpret_cast<tmk::ModelPoint*>(vp);
        if (e == hipSuccess)
            e = hipMemcpy(ml.pts, hp.data(), sizeof(tmk::ModelPoint) * ml.n, hipMemcpyHostToDevice);
        vp = nullptr;
        if (e == hipSuccess) e = tmk::dev_alloc(A, &vp, sizeof(double2) * ml.n, s);
        ml.dir = reinterpret_cast<double2*>(vp);
        if (e == hipSuccess) e = tmk::launch_unit_dirs(ml.pts, ml.n, ml.dir, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            tmk::dev_free(A, tmp, s);
            tm_model_free(m);
            return hip_fail(e, "tm_build_model: point copy");
        }
        int r2 = 0;
        for (const auto& q : hp) r2 = std::max(r2, (int)q.tx * q.tx + (int)q.ty * q.ty);
        ml.radius2 = r2;
        // |round(R t)| <= |t| + 1 per component
        ml.rad = (int)ceil(sqrt((double)r2)) + 1;
    }
    tmk::dev_free(A, tmp, s);
    *out = m;
    return TM_OK;
}

TM_EXPORT void tm_model_free(tm_model* m)
{
    if (!m) return;
    for (int l = 0; l < m->L; ++l) {
        tmk::dev_free(m->alloc, m->lv[l].pts, nullptr);
        tmk::dev_free(m->alloc, m->lv[l].dir, nullptr);
    }
    for (tm_rot_table& c : m->tables) {
        tmk::dev_free(m->alloc, c.tab, nullptr);
        if (c.ready) (void)hipEventDestroy(c.ready);
    }
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
    Grid rigid;
    memset(&rigid, 0, sizeof(rigid));
    rigid.S = 1;
    rigid.sigma_min = 1.0;
    rigid.sigma_max = 1.0;
    tm_status st = get_table(m, level, theta_min, step, K, rigid, S(stream), &tab);
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
    if (field && !p->lv[level].field)
        return fail(TM_EINVAL, "tm_pyramid_read: level %d keeps no field in the pyramid's precision "
                               "(a batch's FP16 pyramid keeps FP16 directions at its top level only)", level);
    if (img) HIP_TRY(hipMemcpyAsync(img, p->lv[level].img, np, hipMemcpyDeviceToDevice, S(stream)));
    if (field)
        HIP_TRY(hipMemcpyAsync(field, p->lv[level].field, np * (p->precision == TM_FP16 ? 4 : 8),
                               hipMemcpyDeviceToDevice, S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_score_poses(const tm_model* m, const tm_pyramid* p, int32_t level, int32_t win, int32_t vote,
                                   const tm_eval_pose* poses, int32_t n, float* scores, void* stream)
{
    tm_status st = check_pair(m, p, "tm_score_poses");
    if (st != TM_OK) return st;
    if (level < 0 || level >= p->L) return fail(TM_EINVAL, "tm_score_poses: bad level %d", level);
    if (win < 1 || win % 2 == 0 || win > 31) return fail(TM_EINVAL, "tm_score_poses: window must be odd in [1, 31]");
    if (vote != TM_VOTE_ALL && vote != TM_VOTE_EDGE)
        return fail(TM_EINVAL, "tm_score_poses: vote must be TM_VOTE_ALL or TM_VOTE_EDGE");
    if (n < 0) return fail(TM_EINVAL, "tm_score_poses: n < 0");
    if (n > 0 && (!poses || !scores)) return fail(TM_EINVAL, "tm_score_poses: null buffer");
    if (!p->lv[level].field)
        return fail(TM_EINVAL, "tm_score_poses: level %d keeps no field in the pyramid's precision", level);
    HIP_TRY(tmk::launch_sparse(p->lv[level].field, p->lv[level].w, p->lv[level].h, p->precision, m->lv[level].pts,
                              m->lv[level].n, win, vote, poses, n, scores, S(stream)));
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
    if (!p->lv[level].field)
        return fail(TM_EINVAL, "tm_score_map: level %d keeps no field in the pyramid's precision", level);
    if (!sw || !s1 || !k) return fail(TM_EINVAL, "tm_score_map: null output");
    Grid g;
    st = make_grid(sp, p->L, &g);
    if (st != TM_OK) return st;
    hipStream_t s = S(stream);
    const tmk::TabEntry* tab = nullptr;
    st = get_table(m, level, sp->theta_min_deg, g.step[level], g.K[level], g, s, &tab);
    if (st != TM_OK) return st;
    tmk::SearchDesc sd = make_search(sp, g, level, p->precision, 1);
    tmk::PairGeom pg = pair_geom(m, p, level, sp->step_x, sp->step_y, g.sigma_max);
    tmk::DensePlan plan = tmk::plan_dense(sd, &pg, 1);
    tmk::PairDesc d;
    memset(&d, 0, sizeof(d));
    pair_static(&d, m, p, tab, level, pg, plan, 0.f, sp->neighbourhood, g.sigma_max);
    st = ensure_ws(p, kDescBytes + pair_scratch(&d, m, pg, plan, p->L, 1, true, false, false, nullptr), s);
    if (st != TM_OK) return st;
    pair_scratch(&d, m, pg, plan, p->L, 1, true, false, false, reinterpret_cast<uint8_t*>(p->ws.ptr) + kDescBytes);
    d.mw = sw;
    d.m1 = s1;
    d.mk = k;
    tmk::PairDesc* dd = nullptr;
    st = put_desc(p, d, s, &dd);
    if (st != TM_OK) return st;
    hipEvent_t ev0, ev1;
    st = timing_pair(&ev0, &ev1);
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_dense(sd, plan, dd, 1, s, ev0, ev1));
    return TM_OK;
}

TM_EXPORT tm_status tm_select(const float* sw, const float* s1, const int32_t* k, int32_t gw, int32_t gh,
                              int32_t sx, int32_t sy, int32_t level, float min_score, float dmin, tm_pose* out,
                              int32_t capacity, int32_t* n_out, void* stream)
{
    if (!sw || !s1 || !k || !out || !n_out) return fail(TM_EINVAL, "tm_select: null argument");
    if (gw < 1 || gh < 1 || sx < 1 || sy < 1 || level < 0 || level >= 31)
        return fail(TM_EINVAL, "tm_select: bad geometry");
    if ((long long)gw * gh > (1LL << 28)) return fail(TM_EINVAL, "tm_select: map too large");
    if (capacity < 1 || capacity > 1024) return fail(TM_EINVAL, "tm_select: capacity must be in [1, 1024]");
    if (!isfinite(min_score) || !isfinite(dmin)) return fail(TM_EINVAL, "tm_select: non-finite threshold");
    // scratch: a private buffer of this thread (this entry point has no
    // pyramid), with the allocator it came from
    static thread_local void* sel_buf = nullptr;
    static thread_local size_t sel_bytes = 0;
    static thread_local tm_allocator sel_alloc = {nullptr, nullptr, nullptr};
    const size_t need = kDescBytes + tmk::select_scratch_bytes(gw * gh);
    hipStream_t s = S(stream);
    if (need > sel_bytes) {
        if (sel_buf) {
            HIP_TRY(hipStreamSynchronize(s));
            tmk::dev_free(sel_alloc, sel_buf, s);
            sel_buf = nullptr;
            sel_bytes = 0;
        }
        sel_alloc = current_allocator();
        HIP_TRY(tmk::dev_alloc(sel_alloc, &sel_buf, need, s));
        sel_bytes = need;
    }
    tmk::SearchDesc sd;
    memset(&sd, 0, sizeof(sd));
    sd.L = level + 1;
    sd.level = level;
    sd.sx = sx;
    sd.sy = sy;
    sd.min_score = min_score;
    sd.max_cand = capacity;
    tmk::PairDesc d;
    memset(&d, 0, sizeof(d));
    d.gw = gw;
    d.gh = gh;
    d.dmin = dmin;
    d.mw = const_cast<float*>(sw);
    d.m1 = const_cast<float*>(s1);
    d.mk = const_cast<int32_t*>(k);
    d.sel = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(sel_buf) + kDescBytes);
    d.cand = out;
    d.ncand = n_out;
    tmk::PairDesc* dd = reinterpret_cast<tmk::PairDesc*>(sel_buf);
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, dd);
    HIP_TRY(hipGetLastError());
    HIP_TRY(tmk::launch_select(sd, dd, 1, gw * gh, s));
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
    st = get_table(m, top, sp->theta_min_deg, g.step[top], g.K[top], g, s, &tab);
    if (st != TM_OK) return st;
    tmk::SearchDesc sd = make_search(sp, g, top, p->precision, capacity);
    sd.screen = p->precision == TM_FP16;  // an FP16 search is a screen whose decisions are certified
    tmk::PairGeom pg = pair_geom(m, p, top, sp->step_x, sp->step_y, g.sigma_max);
    tmk::DensePlan plan = tmk::plan_dense(sd, &pg, 1);
    tmk::PairDesc d;
    memset(&d, 0, sizeof(d));
    pair_static(&d, m, p, tab, top, pg, plan, default_dmin(m, sp), sp->neighbourhood, g.sigma_max);
    const bool refine = p->L > 1;
    const bool certify = plan.screen;
    const size_t pair_bytes = pair_scratch(&d, m, pg, plan, p->L, sp->max_candidates, true, true, refine, nullptr);
    st = ensure_ws(p, kDescBytes + pair_bytes + (certify ? tmk::cert_bytes(pg.gw * pg.gh) : 0), s);
    if (st != TM_OK) return st;
    pair_scratch(&d, m, pg, plan, p->L, sp->max_candidates, true, true, refine,
                 reinterpret_cast<uint8_t*>(p->ws.ptr) + kDescBytes);
    // the outputs go to the final kernel as arguments, so the descriptor (and
    // its device copy) stays the same across calls that write elsewhere
    tmk::PairDesc* dd = nullptr;
    st = put_desc(p, d, s, &dd);
    if (st != TM_OK) return st;
    hipEvent_t ev0, ev1;
    st = timing_pair(&ev0, &ev1);
    if (st != TM_OK) return st;
    const tmk::CertBufs cb =
        tmk::cert_bufs(reinterpret_cast<uint8_t*>(p->ws.ptr) + kDescBytes + pair_bytes, pg.gw * pg.gh);
    HIP_TRY(tmk::launch_dense(sd, plan, dd, 1, s, ev0, ev1, certify ? cb.count : nullptr));
    if (certify) HIP_TRY(tmk::launch_certify(sd, plan, dd, 1, cb, s, true));
    HIP_TRY(tmk::launch_select(sd, dd, 1, pg.gw * pg.gh, s));
    if (refine) {
        const tmk::RefinePlan rp =
            refine_plan(&m, 1, p->L, sp->neighbourhood, sp->max_candidates, g.sigma_max);
        HIP_TRY(tmk::launch_refine(sd, dd, 1, top, rp, s, false));
    }
    HIP_TRY(tmk::launch_final(sd, dd, 1, s, out, n_out, refine ? top % 2 : -1));
    return TM_OK;
}

// ---------------------------------------------------------------- no allocation
// tm_detect_static: every scratch buffer of a detection in this array, one
// copy per GPU, held until the process ends.  Host code never uses the name
// (on the host it is a stand-in, not a device address): each device's
// address comes from hipGetSymbolAddress, once, and is kept in g_static_ptr.
static __device__ __align__(256) unsigned char scratch[TM_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

tm_status static_scratch(void** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TM_EDEVICE, "tm_detect_static: device %d out of range", dev);
    std::lock_guard<std::mutex> g(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                     "tm_detect_static: hipGetSymbolAddress");
        g_static_ptr[dev] = ptr;
    }
    *out = g_static_ptr[dev];
    return TM_OK;
}
}  // namespace

TM_EXPORT tm_status tm_detect_static(const tm_model* m, const tm_pyramid* p, const tm_search_params* sp,
                                     tm_pose* out, int32_t capacity, int32_t* n_out, void* stream)
{
    tm_status st = check_pair(m, p, "tm_detect_static");
    if (st != TM_OK) return st;
    st = check_search(sp, "tm_detect_static");
    if (st != TM_OK) return st;
    if (!out || !n_out) return fail(TM_EINVAL, "tm_detect_static: null output");
    if (capacity < 1) return fail(TM_EINVAL, "tm_detect_static: capacity < 1");
    Grid g;
    st = make_grid(sp, p->L, &g);
    if (st != TM_OK) return st;
    hipStream_t s = S(stream);
    const int top = p->L - 1;
    const tm_model_level& mt = m->lv[top];
    if (scaled_rad(mt, g.sigma_max) > 32000) return fail(TM_EINVAL, "tm_detect_static: model too large for the scale range");
    tmk::SearchDesc sd = make_search(sp, g, top, p->precision, capacity);
    sd.screen = p->precision == TM_FP16;
    tmk::PairGeom pg = pair_geom(m, p, top, sp->step_x, sp->step_y, g.sigma_max);
    tmk::DensePlan plan = tmk::plan_dense(sd, &pg, 1);
    tmk::PairDesc d;
    memset(&d, 0, sizeof(d));
    const bool refine = p->L > 1;
    // layout: descriptor, rotated table of the top level, pair scratch
    const size_t tab_bytes = align_up((size_t)g.K[top] * g.S * mt.n_pad * sizeof(tmk::TabEntry), 256);
    const bool certify = plan.screen;
    const size_t pair_bytes = pair_scratch(&d, m, pg, plan, p->L, sp->max_candidates, true, true, refine, nullptr);
    const size_t need = kDescBytes + tab_bytes + pair_bytes + (certify ? tmk::cert_bytes(pg.gw * pg.gh) : 0);
    if (need > (size_t)TM_STATIC_SCRATCH_BYTES)
        return fail(TM_ECAPACITY, "tm_detect_static: the detection needs %zu bytes of scratch, the static array "
                                  "holds %zu", need, (size_t)TM_STATIC_SCRATCH_BYTES);
    void* base = nullptr;
    st = static_scratch(&base);
    if (st != TM_OK) return st;
    uint8_t* b = reinterpret_cast<uint8_t*>(base);
    tmk::TabEntry* tab = reinterpret_cast<tmk::TabEntry*>(b + kDescBytes);
    HIP_TRY(tmk::launch_tables(mt.pts, mt.n, mt.n_pad, sp->theta_min_deg, g.step[top], g.K[top], g.sigma_min,
                               g.sigma_step, g.S, tab, s));
    pair_static(&d, m, p, tab, top, pg, plan, default_dmin(m, sp), sp->neighbourhood, g.sigma_max);
    pair_scratch(&d, m, pg, plan, p->L, sp->max_candidates, true, true, refine, b + kDescBytes + tab_bytes);
    tmk::PairDesc* dd = reinterpret_cast<tmk::PairDesc*>(b);
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, dd);
    HIP_TRY(hipGetLastError());
    const tmk::CertBufs cb = tmk::cert_bufs(b + kDescBytes + tab_bytes + pair_bytes, pg.gw * pg.gh);
    HIP_TRY(tmk::launch_dense(sd, plan, dd, 1, s, nullptr, nullptr, certify ? cb.count : nullptr));
    if (certify) HIP_TRY(tmk::launch_certify(sd, plan, dd, 1, cb, s, true));
    HIP_TRY(tmk::launch_select(sd, dd, 1, pg.gw * pg.gh, s));
    if (refine) {
        const tmk::RefinePlan rp =
            refine_plan(&m, 1, p->L, sp->neighbourhood, sp->max_candidates, g.sigma_max);
        HIP_TRY(tmk::launch_refine(sd, dd, 1, top, rp, s, false));
    }
    HIP_TRY(tmk::launch_final(sd, dd, 1, s, out, n_out, refine ? top % 2 : -1));
    return TM_OK;
}

TM_EXPORT tm_status tm_probe(int32_t kind, int32_t iterations, void* buf, int64_t buf_bytes, void* stream,
                             double* work)
{
    if (kind < 0 || kind > 6) return fail(TM_EINVAL, "tm_probe: kind must be 0..6");
    if (iterations < 1 || iterations > 1000000) return fail(TM_EINVAL, "tm_probe: iterations must be 1..10^6");
    if (!buf || buf_bytes < 256 || !work) return fail(TM_EINVAL, "tm_probe: need a buffer of >= 256 bytes");
    HIP_TRY(tmk::launch_probe(kind, iterations, buf, buf_bytes, S(stream), work));
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
    if (from_level < 0 || from_level >= p->L) return fail(TM_EINVAL, "tm_refine: bad from_level %d", from_level);
    if (n == 0) return TM_OK;
    if (!poses) return fail(TM_EINVAL, "tm_refine: null poses");
    Grid g;
    st = make_grid(sp, p->L, &g);
    if (st != TM_OK) return st;
    if (from_level == 0) return TM_OK;
    hipStream_t s = S(stream);
    tmk::SearchDesc sd = make_search(sp, g, from_level, p->precision, 1);
    sd.max_cand = n;
    tmk::PairGeom pg = pair_geom(m, p, from_level, sp->step_x, sp->step_y, g.sigma_max);
    tmk::DensePlan plan = {};
    tmk::PairDesc d;
    memset(&d, 0, sizeof(d));
    pair_static(&d, m, p, nullptr, from_level, pg, plan, 0.f, sp->neighbourhood, g.sigma_max);
    st = ensure_ws(p, kDescBytes + pair_scratch(&d, m, pg, plan, p->L, n, false, false, true, nullptr), s);
    if (st != TM_OK) return st;
    pair_scratch(&d, m, pg, plan, p->L, n, false, false, true, reinterpret_cast<uint8_t*>(p->ws.ptr) + kDescBytes);
    d.cand = poses;
    d.ncand = nullptr;
    tmk::PairDesc* dd = nullptr;
    st = put_desc(p, d, s, &dd);
    if (st != TM_OK) return st;
    const tmk::RefinePlan rp = refine_plan(&m, 1, p->L, sp->neighbourhood, n, g.sigma_max);
    HIP_TRY(tmk::launch_refine(sd, dd, 1, from_level, rp, s));
    return TM_OK;
}

// ======================================================================= continuous

namespace {
// Descriptor of one (model, pyramid) pair for the continuous score, at the
// start of the pyramid's scratch; extra bytes follow it.
tm_status cont_prepare(const tm_model* m, tm_pyramid* p, int level, size_t extra, hipStream_t s,
                       tmk::PairDesc** dd, const char* what)
{
    tm_status st = check_pair(m, p, what);
    if (st != TM_OK) return st;
    if (level < 0 || level >= p->L) return fail(TM_EINVAL, "%s: bad level %d", what, level);
    if (!p->lv[level].field) return fail(TM_EINVAL, "%s: level %d keeps no field in the pyramid's precision", what, level);
    st = ensure_ws(p, kDescBytes + extra, s);
    if (st != TM_OK) return st;
    tmk::PairDesc d;
    memset(&d, 0, sizeof(d));
    for (int l = 0; l < p->L; ++l) {
        d.field[l] = p->lv[l].field;
        d.W[l] = p->lv[l].w;
        d.H[l] = p->lv[l].h;
        d.pts[l] = m->lv[l].pts;
        d.dir[l] = m->lv[l].dir;
        d.n[l] = m->lv[l].n;
    }
    return put_desc(p, d, s, dd);
}
}  // namespace

TM_EXPORT tm_status tm_cont_score(const tm_model* m, tm_pyramid* p, int32_t level, const tm_cont_pose* poses,
                                  int32_t n, float* scores, void* stream)
{
    if (n < 0) return fail(TM_EINVAL, "tm_cont_score: n < 0");
    if (n > 0 && (!poses || !scores)) return fail(TM_EINVAL, "tm_cont_score: null buffer");
    tmk::PairDesc* dd = nullptr;
    tm_status st = cont_prepare(m, p, level, 0, S(stream), &dd, "tm_cont_score");
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_cont(dd, 0, 1, level, p->precision, poses, n, nullptr, scores, false, S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_cont_score_backward(const tm_model* m, tm_pyramid* p, int32_t level,
                                           const tm_cont_pose* poses, int32_t n, const float* gin, float* gout,
                                           void* stream)
{
    if (n < 0) return fail(TM_EINVAL, "tm_cont_score_backward: n < 0");
    if (n > 0 && (!poses || !gout)) return fail(TM_EINVAL, "tm_cont_score_backward: null buffer");
    tmk::PairDesc* dd = nullptr;
    tm_status st = cont_prepare(m, p, level, 0, S(stream), &dd, "tm_cont_score_backward");
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_cont(dd, 0, 1, level, p->precision, poses, n, gin, gout, true, S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_cont_line_search(const tm_model* m, tm_pyramid* p, int32_t level, tm_cont_pose* poses,
                                        const float* dirs, int32_t n, const double* alphas, int32_t n_alphas,
                                        float* scores, void* stream)
{
    if (n < 0) return fail(TM_EINVAL, "tm_cont_line_search: n < 0");
    if (n > 0 && (!poses || !dirs)) return fail(TM_EINVAL, "tm_cont_line_search: null buffer");
    if (!alphas || n_alphas < 1 || n_alphas > 16)
        return fail(TM_EINVAL, "tm_cont_line_search: need 1..16 step lengths");
    for (int j = 0; j < n_alphas; ++j)
        if (!isfinite(alphas[j])) return fail(TM_EINVAL, "tm_cont_line_search: non-finite step length");
    if ((long long)n * n_alphas > (1LL << 30)) return fail(TM_EINVAL, "tm_cont_line_search: too many evaluations");
    tmk::PairDesc* dd = nullptr;
    tm_status st = cont_prepare(m, p, level, tmk::line_search_scratch_bytes(n, n_alphas), S(stream), &dd,
                                "tm_cont_line_search");
    if (st != TM_OK) return st;
    double* ls_scratch = reinterpret_cast<double*>(reinterpret_cast<uint8_t*>(p->ws.ptr) + kDescBytes);
    HIP_TRY(tmk::launch_line_search(dd, 0, 1, level, p->precision, poses, dirs, n, alphas, n_alphas, scores, ls_scratch,
                                    S(stream)));
    return TM_OK;
}

// ======================================================================= batch

struct tm_batch_s {
    int n_models = 0, n_images = 0, npairs = 0, L = 0;
    std::vector<tm_pyramid*> pyrs;
    std::vector<const tm_model*> models;
    tmk::SearchDesc sd;
    tmk::DensePlan plan;
    tmk::RefinePlan rplan;
    int level_w[TM_MAX_LEVELS], level_h[TM_MAX_LEVELS];
    int max_field_blocks = 0, max_np = 0;
    void* scratch = nullptr;
    tmk::PairDesc* d_pairs = nullptr;
    tmk::PyrBuildArg* d_pb = nullptr;
    tmk::FieldsArg* d_fa = nullptr;
    hipGraphExec_t graph = nullptr;  // captured tm_batch_run, made by the first tm_batch_run_graph
    void* ls_buf = nullptr;          // line-search scratch of the continuous score
    size_t ls_bytes = 0;
    tm_allocator alloc = {};         // allocator of the batch's memory
    hipEvent_t last_run = nullptr;   // recorded after each run enqueued outside a capture
    bool certify = false;            // FP16 search: its decisions are certified in FP32
    tmk::CertBufs cert = {};
    // what a change of the search's angle chunking needs: the pairs' geometry,
    // the host copies of their descriptors, their scratch regions (sized for
    // the largest chunking offered), and the work list's room
    std::vector<tmk::PairGeom> pg;
    std::vector<tmk::PairDesc> hd;
    std::vector<size_t> pair_off;
    uint8_t* base = nullptr;
    int2* work_dev = nullptr;
    size_t work_cap = 0;
    int c_max = 1;                   // most angle chunks the scratch holds
    int max_cand = 0;
    bool refine = false;
};

namespace {
// Wait until the device has passed the batch's last run (before its graph is
// replaced, its scratch reused by the tuner, or its memory freed).
tm_status batch_wait(tm_batch* b)
{
    if (b->last_run) HIP_TRY(hipEventSynchronize(b->last_run));
    return TM_OK;
}
}  // namespace

TM_EXPORT void tm_batch_free(tm_batch* b)
{
    if (!b) return;
    (void)batch_wait(b);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    tmk::dev_free(b->alloc, b->ls_buf, nullptr);
    for (tm_pyramid* p : b->pyrs) tm_pyramid_free(p);
    tmk::dev_free(b->alloc, b->scratch, nullptr);
    if (b->last_run) (void)hipEventDestroy(b->last_run);
    delete b;
}

TM_EXPORT tm_status tm_batch_create(const tm_model* const* models, int32_t n_models, const uint8_t* const* images,
                                    const int32_t* widths, const int32_t* heights, const int32_t* pitches,
                                    int32_t n_images, const tm_pyr_params* pp, const tm_search_params* sp,
                                    tm_pose* out, int32_t capacity, int32_t* n_out, void* stream, tm_batch** outb)
{
    g_err[0] = 0;
    if (!outb) return fail(TM_EINVAL, "tm_batch_create: null out");
    *outb = nullptr;
    if (!models || !images || !widths || !heights || !pitches || !pp || !out || !n_out)
        return fail(TM_EINVAL, "tm_batch_create: null argument");
    if (n_models < 1 || n_images < 1) return fail(TM_EINVAL, "tm_batch_create: need at least one model and image");
    if ((long long)n_models * n_images > 65535) return fail(TM_EINVAL, "tm_batch_create: more than 65535 pairs");
    if (capacity < 1) return fail(TM_EINVAL, "tm_batch_create: capacity < 1");
    tm_status st = check_search(sp, "tm_batch_create");
    if (st != TM_OK) return st;
    for (int j = 0; j < n_models; ++j) {
        if (!models[j]) return fail(TM_EINVAL, "tm_batch_create: null model %d", j);
        if (models[j]->L < pp->levels)
            return fail(TM_EINVAL, "tm_batch_create: model %d has %d levels, need %d", j, models[j]->L, pp->levels);
    }
    for (int i = 0; i < n_images; ++i) {
        st = check_image(images[i], widths[i], heights[i], pitches[i], pp, "tm_batch_create");
        if (st != TM_OK) return st;
    }
    const int L = pp->levels, top = L - 1;
    Grid g;
    st = make_grid(sp, L, &g);
    if (st != TM_OK) return st;
    hipStream_t s = S(stream);
    tm_batch* b = new (std::nothrow) tm_batch_s();
    if (!b) return fail(TM_ENOMEM, "tm_batch_create: host allocation");
    b->alloc = current_allocator();
    if (hipEventCreateWithFlags(&b->last_run, hipEventDisableTiming) != hipSuccess) {
        b->last_run = nullptr;
        tm_batch_free(b);
        return fail(TM_EDEVICE, "tm_batch_create: hipEventCreate");
    }
    b->n_models = n_models;
    b->n_images = n_images;
    b->npairs = n_models * n_images;
    b->L = L;
    b->models.assign(models, models + n_models);
    for (int i = 0; i < n_images; ++i) {
        tm_pyramid* p = nullptr;
        st = alloc_pyramid(widths[i], heights[i], pp, s, &p, true);
        if (st != TM_OK) {
            tm_batch_free(b);
            return st;
        }
        b->pyrs.push_back(p);
    }
    b->sd = make_search(sp, g, top, pp->precision, capacity);
    b->sd.screen = pp->precision == TM_FP16;
    std::vector<tmk::PairGeom> pg(b->npairs);
    for (int i = 0; i < n_images; ++i)
        for (int j = 0; j < n_models; ++j)
            pg[i * n_models + j] = pair_geom(models[j], b->pyrs[i], top, sp->step_x, sp->step_y, g.sigma_max);
    b->plan = tmk::plan_dense(b->sd, pg.data(), b->npairs);
    std::vector<int2> work;
    if (!tmk::build_work(b->plan, pg.data(), b->npairs, work)) {
        tm_batch_free(b);
        return fail(TM_EDEVICE, "tm_batch_create: internal error in the search work list");
    }
    // the autotuner may choose another angle chunking: up to four times the
    // planned number of chunks (at most 12), whose scratch and work list are
    // sized here
    tmk::DensePlan plan_max = b->plan;
    b->c_max = b->plan.C;
    size_t work_cap = work.size();
    if (b->plan.fast) {
        b->c_max = std::max(b->plan.C, std::min(12, 4 * b->plan.C));
        for (int A : tmk::chunk_candidates(b->plan, b->sd, b->c_max)) {
            tmk::DensePlan q = b->plan;
            std::vector<int2> w;
            if (!tmk::rechunk_dense(q, b->sd, pg.data(), b->npairs, A) || !tmk::build_work(q, pg.data(), b->npairs, w)) {
                tm_batch_free(b);
                return fail(TM_EDEVICE, "tm_batch_create: internal error in the search work list");
            }
            work_cap = std::max(work_cap, w.size());
            if (q.C > plan_max.C) plan_max = q;
        }
    }
    b->work_cap = work_cap;
    b->rplan = refine_plan(models, n_models, L, sp->neighbourhood,
                           (long long)b->npairs * sp->max_candidates, g.sigma_max);
    for (auto& q : pg) b->max_np = std::max(b->max_np, q.gw * q.gh);

    // one allocation: tables, descriptors, pyramid arguments, pair scratch
    const int K = g.K[top];
    for (int j = 0; j < n_models; ++j)
        if (scaled_rad(models[j]->lv[top], g.sigma_max) > 32000) {
            tm_batch_free(b);
            return fail(TM_EINVAL, "tm_batch_create: model too large for the scale range");
        }
    std::vector<size_t> tab_off(n_models);
    size_t off = 0;
    for (int j = 0; j < n_models; ++j) {
        tab_off[j] = off;
        off = align_up(off + (size_t)K * g.S * models[j]->lv[top].n_pad * sizeof(tmk::TabEntry), 256);
    }
    const size_t desc_off = off;
    off = align_up(off + (size_t)b->npairs * sizeof(tmk::PairDesc), 256);
    const size_t pb_off = off;
    off = align_up(off + (size_t)n_images * sizeof(tmk::PyrBuildArg), 256);
    const size_t fa_off = off;
    off = align_up(off + (size_t)n_images * sizeof(tmk::FieldsArg), 256);
    const size_t work_off = off;
    off = align_up(off + work_cap * sizeof(int2), 256);
    long long total_np = 0;
    for (auto& q : pg) total_np += (long long)q.gw * q.gh;
    if (total_np > (1LL << 30)) {
        tm_batch_free(b);
        return fail(TM_EINVAL, "tm_batch_create: too many translations");
    }
    b->certify = b->plan.screen;
    const size_t cert_off = off;
    if (b->certify) off = align_up(off + tmk::cert_bytes((int)total_np), 256);
    std::vector<size_t> pair_off(b->npairs);
    const bool refine = L > 1;
    for (int q = 0; q < b->npairs; ++q) {
        tmk::PairDesc tmp;
        memset(&tmp, 0, sizeof(tmp));
        pair_off[q] = off;
        off += align_up(pair_scratch(&tmp, models[q % n_models], pg[q], plan_max, L, sp->max_candidates, true, true,
                                     refine, nullptr),
                        256);
    }
    hipError_t e = tmk::dev_alloc(b->alloc, &b->scratch, off, s);
    if (e != hipSuccess) {
        tm_batch_free(b);
        return hip_fail(e, "tm_batch_create: device allocation");
    }
    uint8_t* base = reinterpret_cast<uint8_t*>(b->scratch);
    b->d_pairs = reinterpret_cast<tmk::PairDesc*>(base + desc_off);
    if (b->certify) b->cert = tmk::cert_bufs(base + cert_off, (int)total_np);
    b->d_pb = reinterpret_cast<tmk::PyrBuildArg*>(base + pb_off);
    b->d_fa = reinterpret_cast<tmk::FieldsArg*>(base + fa_off);
    for (int j = 0; j < n_models; ++j) {
        const tm_model_level& ml = models[j]->lv[top];
        e = tmk::launch_tables(ml.pts, ml.n, ml.n_pad, sp->theta_min_deg, g.step[top], K, g.sigma_min, g.sigma_step,
                               g.S, reinterpret_cast<tmk::TabEntry*>(base + tab_off[j]), s);
        if (e != hipSuccess) {
            tm_batch_free(b);
            return hip_fail(e, "tm_batch_create: tables");
        }
    }
    std::vector<tmk::PairDesc> hd(b->npairs);
    for (int i = 0; i < n_images; ++i)
        for (int j = 0; j < n_models; ++j) {
            const int q = i * n_models + j;
            tmk::PairDesc& d = hd[q];
            memset(&d, 0, sizeof(d));
            pair_static(&d, models[j], b->pyrs[i], reinterpret_cast<tmk::TabEntry*>(base + tab_off[j]), top, pg[q],
                        b->plan, default_dmin(models[j], sp), sp->neighbourhood, g.sigma_max);
            pair_scratch(&d, models[j], pg[q], b->plan, L, sp->max_candidates, true, true, refine,
                         base + pair_off[q]);
            d.out = out + (size_t)q * capacity;
            d.n_out = n_out + q;
        }
    std::vector<tmk::PyrBuildArg> hpb(n_images);
    std::vector<tmk::FieldsArg> hfa(n_images);
    for (int l = 0; l < L; ++l) b->level_w[l] = b->level_h[l] = 0;
    for (int i = 0; i < n_images; ++i) {
        hpb[i] = tmk::pyr_build_arg(images[i], pitches[i], b->pyrs[i]->lv, L);
        hfa[i] = tmk::fields_arg(b->pyrs[i]->lv, L, b->pyrs[i]->T2, pp->precision);
        b->max_field_blocks = std::max(b->max_field_blocks, hfa[i].block0[L]);
        for (int l = 0; l < L; ++l) {
            b->level_w[l] = std::max(b->level_w[l], b->pyrs[i]->lv[l].w);
            b->level_h[l] = std::max(b->level_h[l], b->pyrs[i]->lv[l].h);
        }
    }
    e = hipMemcpyAsync(b->d_pairs, hd.data(), hd.size() * sizeof(tmk::PairDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_pb, hpb.data(), hpb.size() * sizeof(tmk::PyrBuildArg), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_fa, hfa.data(), hfa.size() * sizeof(tmk::FieldsArg), hipMemcpyHostToDevice, s);
    b->work_dev = reinterpret_cast<int2*>(base + work_off);
    if (e == hipSuccess && !work.empty()) {
        b->plan.work = b->work_dev;
        b->plan.n_work = (int)work.size();
        e = hipMemcpyAsync(base + work_off, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        tm_batch_free(b);
        return hip_fail(e, "tm_batch_create: upload");
    }
    b->pg = pg;
    b->hd = hd;
    b->pair_off = pair_off;
    b->base = base;
    b->max_cand = sp->max_candidates;
    b->refine = refine;
    *outb = b;
    return TM_OK;
}

namespace {
// Give the batch a plan with another angle chunking (and form): the pairs'
// scratch pointers and the work list follow it.  Waits for the batch's last
// run and for the uploads; the captured graph is discarded.
tm_status batch_apply_plan(tm_batch* b, tmk::DensePlan p, hipStream_t s)
{
    if (p.C > b->c_max) return fail(TM_EINVAL, "angle chunking beyond the batch's scratch (%d chunks, at most %d)",
                                    p.C, b->c_max);
    std::vector<int2> work;
    if (!tmk::build_work(p, b->pg.data(), b->npairs, work) || work.size() > b->work_cap)
        return fail(TM_EDEVICE, "internal error in the search work list");
    tm_status st = batch_wait(b);
    if (st != TM_OK) return st;
    for (int q = 0; q < b->npairs; ++q)
        pair_scratch(&b->hd[q], b->models[q % b->n_models], b->pg[q], p, b->L, b->max_cand, true, true, b->refine,
                     b->base + b->pair_off[q]);
    HIP_TRY(hipMemcpyAsync(b->d_pairs, b->hd.data(), b->hd.size() * sizeof(tmk::PairDesc), hipMemcpyHostToDevice, s));
    p.work = nullptr;
    p.n_work = 0;
    if (!work.empty()) {
        HIP_TRY(hipMemcpyAsync(b->work_dev, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice, s));
        p.work = b->work_dev;
        p.n_work = (int)work.size();
    }
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(tmk::prepare_dense(b->sd, p));
    b->plan = p;
    if (b->graph) {  // captured with the old plan
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return TM_OK;
}
}  // namespace

namespace {
tm_status batch_enqueue(tm_batch* b, hipStream_t s, bool timed)
{
    const int top = b->L - 1;
    HIP_TRY(tmk::launch_pyramids_batch(b->d_pb, b->d_fa, b->n_images, b->L, b->level_w[0], b->level_h[0],
                                       b->max_field_blocks, b->level_w, b->level_h,
                                       b->pyrs[0]->source == TM_PYR_GRADIENT, s));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (timed) {
        tm_status st = timing_pair(&ev0, &ev1);
        if (st != TM_OK) return st;
    }
    HIP_TRY(tmk::launch_dense(b->sd, b->plan, b->d_pairs, b->npairs, s, ev0, ev1,
                              b->certify ? b->cert.count : nullptr));
    if (b->certify) HIP_TRY(tmk::launch_certify(b->sd, b->plan, b->d_pairs, b->npairs, b->cert, s, true));
    HIP_TRY(tmk::launch_select(b->sd, b->d_pairs, b->npairs, b->max_np, s));
    if (b->L > 1) HIP_TRY(tmk::launch_refine(b->sd, b->d_pairs, b->npairs, top, b->rplan, s, false));
    HIP_TRY(tmk::launch_final(b->sd, b->d_pairs, b->npairs, s, nullptr, nullptr, b->L > 1 ? top % 2 : -1));
    return TM_OK;
}
}  // namespace

TM_EXPORT tm_status tm_batch_run(tm_batch* b, void* stream)
{
    if (!b) return fail(TM_EINVAL, "tm_batch_run: null batch");
    const tm_status st = batch_enqueue(b, S(stream), true);
    if (st == TM_OK && !stream_capturing(S(stream))) HIP_TRY(hipEventRecord(b->last_run, S(stream)));
    return st;
}

TM_EXPORT tm_status tm_batch_run_graph(tm_batch* b, void* stream)
{
    if (!b) return fail(TM_EINVAL, "tm_batch_run_graph: null batch");
    if (!b->graph) {
        // Capture on a private stream: nothing runs, the launches become nodes.
        HIP_TRY(tmk::prepare_dense(b->sd, b->plan));
        HIP_TRY(tmk::prepare_refine());
        HIP_TRY(tmk::launch_certify(b->sd, b->plan, nullptr, 0, b->cert, nullptr));  // kernel attributes only
        hipStream_t cs = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        tm_status st = TM_OK;
        if (e == hipSuccess) {
            st = batch_enqueue(b, cs, false);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (st == TM_OK && e2 != hipSuccess) st = hip_fail(e2, "tm_batch_run_graph: end capture");
            if (st == TM_OK) {
                e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    b->graph = nullptr;
                    st = hip_fail(e, "tm_batch_run_graph: instantiate");
                }
            }
            if (g) (void)hipGraphDestroy(g);
        } else {
            st = hip_fail(e, "tm_batch_run_graph: begin capture");
        }
        (void)hipStreamDestroy(cs);
        if (st != TM_OK) return st;
    }
    HIP_TRY(hipGraphLaunch(b->graph, S(stream)));
    if (!stream_capturing(S(stream))) HIP_TRY(hipEventRecord(b->last_run, S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_batch_set_form(tm_batch* b, int32_t variant, int32_t waves, int32_t chunk)
{
    if (!b) return fail(TM_EINVAL, "tm_batch_set_form: null batch");
    if (!b->plan.fast) {
        if (variant == -1) return TM_OK;
        return fail(TM_EINVAL, "tm_batch_set_form: the batch uses the generic search, which has no forms");
    }
    tmk::DensePlan p = b->plan;
    if (!tmk::retune_dense(p, variant, waves))
        return fail(TM_EINVAL, "tm_batch_set_form: variant %d with %d waves per chunk does not apply to this batch",
                    variant, waves);
    if (chunk < 0) return fail(TM_EINVAL, "tm_batch_set_form: chunk must be >= 0");
    if (chunk > 0 && !tmk::rechunk_dense(p, b->sd, b->pg.data(), b->npairs, chunk))
        return fail(TM_EINVAL, "tm_batch_set_form: chunk %d does not apply", chunk);
    if (p.C > b->c_max)
        return fail(TM_EINVAL, "tm_batch_set_form: %d angles a chunk makes %d chunks, the batch holds at most %d", chunk,
                    p.C, b->c_max);
    return batch_apply_plan(b, p, nullptr);
}

TM_EXPORT tm_status tm_batch_search_form(const tm_batch* b, int32_t* variant, int32_t* waves, int32_t* chunk)
{
    if (!b || !variant || !waves) return fail(TM_EINVAL, "tm_batch_search_form: null argument");
    *variant = b->plan.fast ? b->plan.variant : -1;
    *waves = b->plan.fast ? b->plan.WA : 0;
    if (chunk) *chunk = b->plan.A;
    return TM_OK;
}

TM_EXPORT tm_status tm_batch_search_launch(const tm_batch* b, int32_t* workgroups, int32_t* threads)
{
    if (!b || !workgroups || !threads) return fail(TM_EINVAL, "tm_batch_search_launch: null argument");
    const tmk::DensePlan& p = b->plan;
    if (p.fast) {
        *workgroups = p.work ? p.n_work : p.max_blocks * b->npairs;
        *threads = 64 * p.WY * p.WA;
    } else {
        *workgroups = (p.max_np + 255) / 256 * p.C * b->npairs;
        *threads = 256;
    }
    return TM_OK;
}

namespace {
// Mean milliseconds of one search launch of plan p over the batch.
hipError_t time_search(tm_batch* b, const tmk::DensePlan& p, int iterations, hipStream_t s, hipEvent_t e0,
                       hipEvent_t e1, float* ms)
{
    hipError_t e = tmk::prepare_dense(b->sd, p);
    if (e == hipSuccess) e = tmk::launch_dense(b->sd, p, b->d_pairs, b->npairs, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int it = 0; it < iterations && e == hipSuccess; ++it) e = tmk::launch_dense(b->sd, p, b->d_pairs, b->npairs, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e == hipSuccess) *ms /= iterations;
    return e;
}

// Mean milliseconds of one step of two batches run side by side as graph
// launches, the steps alternating between b on s and c on cs (as a caller
// keeping two batches in flight runs them).
tm_status time_pipelined(tm_batch* b, tm_batch* c, int steps, hipStream_t s, hipStream_t cs, hipEvent_t e0,
                         hipEvent_t e1, hipEvent_t ej, float* ms)
{
    tm_status st = tm_batch_run_graph(b, s);  // captures the graphs (outside the timed steps)
    if (st == TM_OK) st = tm_batch_run_graph(c, cs);
    if (st != TM_OK) return st;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipStreamSynchronize(cs));
    HIP_TRY(hipEventRecord(e0, s));
    HIP_TRY(hipStreamWaitEvent(cs, e0, 0));
    for (int i = 0; i < steps && st == TM_OK; ++i) st = tm_batch_run_graph(i % 2 ? c : b, i % 2 ? cs : s);
    if (st != TM_OK) return st;
    HIP_TRY(hipEventRecord(ej, cs));
    HIP_TRY(hipStreamWaitEvent(s, ej, 0));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    *ms /= steps;
    return TM_OK;
}
}  // namespace

TM_EXPORT tm_status tm_batch_tune(tm_batch* b, tm_batch* partner, int32_t iterations, void* stream,
                                  void* partner_stream, int32_t* variant_out, int32_t* waves_out, int32_t* chunk_out,
                                  float* us_out)
{
    if (!b) return fail(TM_EINVAL, "tm_batch_tune: null batch");
    if (iterations < 1 || iterations > 1000) return fail(TM_EINVAL, "tm_batch_tune: iterations must be 1..1000");
    if (partner) {
        bool same = partner != b && partner->npairs == b->npairs && partner->plan.fast == b->plan.fast &&
                    partner->c_max == b->c_max &&
                    tmk::poses_per_translation(partner->sd) == tmk::poses_per_translation(b->sd);
        for (int q = 0; same && q < b->npairs; ++q)
            same = memcmp(&partner->pg[q], &b->pg[q], sizeof(tmk::PairGeom)) == 0;
        if (!same) return fail(TM_EINVAL, "tm_batch_tune: the partner batch is not of the same shape");
        if (S(partner_stream) == S(stream)) return fail(TM_EINVAL, "tm_batch_tune: the partner needs its own stream");
    }
    hipStream_t s = S(stream);
    if (!b->plan.fast) {
        if (variant_out) *variant_out = -1;
        if (waves_out) *waves_out = 0;
        if (chunk_out) *chunk_out = 0;
        if (us_out) *us_out = 0.f;
        return TM_OK;  // the generic search has no forms to choose from
    }
    // the tuner's launches reuse the batch's scratch: no earlier run may still use it
    tm_status st = batch_wait(b);
    if (st == TM_OK && partner) st = batch_wait(partner);
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_pyramids_batch(b->d_pb, b->d_fa, b->n_images, b->L, b->level_w[0], b->level_h[0],
                                       b->max_field_blocks, b->level_w, b->level_h,
                                       b->pyrs[0]->source == TM_PYR_GRADIENT, s));
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    auto done = [&](tm_status r) {
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        return r;
    };
    if (e != hipSuccess) return done(hip_fail(e, "tm_batch_tune: hipEventCreate"));
    // 1. every (variant, waves per chunk) form that fits, its search launches
    //    timed at the planned chunking in two rounds (a form's time is the
    //    smaller of its two), so that a clock drift during the first round
    //    does not decide
    static const int kWaves[] = {2, 4, 8, 16};
    constexpr int kRounds = 2;
    std::vector<tmk::DensePlan> forms;
    for (int v = 0; v <= 5; ++v)
        for (int wa : kWaves) {
            tmk::DensePlan p = b->plan;
            if (tmk::retune_dense(p, v, wa)) forms.push_back(p);
        }
    std::vector<float> form_ms(forms.size(), INFINITY);
    for (int round = 0; round < kRounds && e == hipSuccess; ++round)
        for (size_t f = 0; f < forms.size() && e == hipSuccess; ++f) {
            float ms = 0.f;
            e = time_search(b, forms[f], iterations, s, ev[0], ev[1], &ms);
            if (e == hipSuccess) form_ms[f] = std::min(form_ms[f], ms);
        }
    if (e != hipSuccess) return done(hip_fail(e, "tm_batch_tune"));
    // 2. the two fastest forms at every angle chunking the batch holds,
    //    timed on the pipelined step of the two batches when a partner is
    //    given (the step is what such a caller sees), else on the search
    std::vector<size_t> order(forms.size());
    for (size_t f = 0; f < order.size(); ++f) order[f] = f;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return form_ms[x] < form_ms[y]; });
    const std::vector<int> chunks = tmk::chunk_candidates(b->plan, b->sd, b->c_max);
    tmk::DensePlan best = forms[order[0]];
    float best_ms = INFINITY;
    for (size_t oi = 0; oi < std::min<size_t>(2, order.size()); ++oi)
        for (int A : chunks) {
            tmk::DensePlan p = forms[order[oi]];
            if (!tmk::rechunk_dense(p, b->sd, b->pg.data(), b->npairs, A) || p.C > b->c_max) continue;
            float ms = 0.f;
            if (partner) {
                st = batch_apply_plan(b, p, s);
                if (st == TM_OK) st = batch_apply_plan(partner, p, S(partner_stream));
                if (st == TM_OK)
                    st = time_pipelined(b, partner, 2 * iterations + 2, s, S(partner_stream), ev[0], ev[1], ev[2], &ms);
                if (st != TM_OK) return done(st);
            } else {
                st = batch_apply_plan(b, p, s);
                if (st != TM_OK) return done(st);
                e = time_search(b, b->plan, iterations, s, ev[0], ev[1], &ms);
                if (e != hipSuccess) return done(hip_fail(e, "tm_batch_tune"));
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = b->plan;
            }
        }
    st = batch_apply_plan(b, best, s);
    if (st == TM_OK && partner) st = batch_apply_plan(partner, best, S(partner_stream));
    if (st != TM_OK) return done(st);
    if (variant_out) *variant_out = best.variant;
    if (waves_out) *waves_out = best.WA;
    if (chunk_out) *chunk_out = best.A;
    if (us_out) *us_out = best_ms * 1000.f;
    return done(TM_OK);
}

namespace {
tm_status batch_cont_check(const tm_batch* b, int level, int n, const void* poses, const void* out, const char* what)
{
    if (!b) return fail(TM_EINVAL, "%s: null batch", what);
    if (level < 0 || level >= b->L) return fail(TM_EINVAL, "%s: bad level %d", what, level);
    if (n < 0) return fail(TM_EINVAL, "%s: n < 0", what);
    if (n > 0 && (!poses || !out)) return fail(TM_EINVAL, "%s: null buffer", what);
    return TM_OK;
}
}  // namespace

TM_EXPORT tm_status tm_batch_cont_score(tm_batch* b, int32_t level, const tm_cont_pose* poses, int32_t n,
                                        float* scores, void* stream)
{
    tm_status st = batch_cont_check(b, level, n, poses, scores, "tm_batch_cont_score");
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_cont(b->d_pairs, 1, b->npairs, level, TM_FP32, poses, n, nullptr, scores, false,
                             S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_batch_cont_score_backward(tm_batch* b, int32_t level, const tm_cont_pose* poses, int32_t n,
                                                 const float* gin, float* gout, void* stream)
{
    tm_status st = batch_cont_check(b, level, n, poses, gout, "tm_batch_cont_score_backward");
    if (st != TM_OK) return st;
    HIP_TRY(tmk::launch_cont(b->d_pairs, 1, b->npairs, level, TM_FP32, poses, n, gin, gout, true, S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_batch_cont_line_search(tm_batch* b, int32_t level, tm_cont_pose* poses, const float* dirs,
                                              int32_t n, const double* alphas, int32_t n_alphas, float* scores,
                                              void* stream)
{
    tm_status st = batch_cont_check(b, level, n, poses, dirs, "tm_batch_cont_line_search");
    if (st != TM_OK) return st;
    if (!alphas || n_alphas < 1 || n_alphas > 16)
        return fail(TM_EINVAL, "tm_batch_cont_line_search: need 1..16 step lengths");
    for (int j = 0; j < n_alphas; ++j)
        if (!isfinite(alphas[j])) return fail(TM_EINVAL, "tm_batch_cont_line_search: non-finite step length");
    if ((long long)n * n_alphas > (1LL << 30))
        return fail(TM_EINVAL, "tm_batch_cont_line_search: too many evaluations");
    const size_t need = tmk::line_search_scratch_bytes(n, n_alphas);
    if (need > b->ls_bytes) {
        if (b->ls_buf) {
            HIP_TRY(hipDeviceSynchronize());  // earlier line searches may still use the buffer
            tmk::dev_free(b->alloc, b->ls_buf, S(stream));
        }
        b->ls_buf = nullptr;
        b->ls_bytes = 0;
        HIP_TRY(tmk::dev_alloc(b->alloc, &b->ls_buf, need, S(stream)));
        b->ls_bytes = need;
    }
    HIP_TRY(tmk::launch_line_search(b->d_pairs, 1, b->npairs, level, TM_FP32, poses, dirs, n, alphas,
                                    n_alphas, scores, reinterpret_cast<double*>(b->ls_buf), S(stream)));
    return TM_OK;
}

TM_EXPORT tm_status tm_batch_pyramid(const tm_batch* b, int32_t image, const tm_pyramid** out)
{
    if (!b || !out) return fail(TM_EINVAL, "tm_batch_pyramid: null argument");
    if (image < 0 || image >= b->n_images) return fail(TM_EINVAL, "tm_batch_pyramid: bad image %d", image);
    *out = b->pyrs[image];
    return TM_OK;
}
