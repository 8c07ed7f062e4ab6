/*
 * Plain FP64 CPU oracle for edge-orientation template matching
 * (Le & Lin, "GPU-accelerated image alignment for object detection in
 * industrial applications", arXiv 2112.05576).
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines what the detector computes, in
 * the most direct form: nested loops, double precision, sums taken in point
 * order, no blocking, no fusion, no reordering.  It shares no code with the
 * HIP library and is used only by the test suite, by the smoke check and by
 * the benchmark's CPU-baseline leg.  Build with -ffp-contract=off so that every
 * product and sum below is rounded exactly as written.
 *
 * Steps and the passages they follow (paper sections / equations):
 *   O1  Sobel gradients                      Sec. II, para. 2 (edge extraction)
 *   O2  magnitude threshold, unit direction  Sec. II, para. 2
 *   O3  image pyramid (2x2 box reduce)       Sec. II, para. 2
 *   O4  model edge points t_i                Sec. II, para. 2 and Eq. (2)
 *   O5  angle grid per level                 Sec. II, para. 2 (step sizes)
 *   O6  rigid projection                     Eq. (2)
 *   O7  windowed similarity score            Eq. (1), Sec. II paras. 3-6
 *   O8  exhaustive (x, y, theta) search      Sec. II, para. 3; Fig. 2
 *   O9  candidates: local max + greedy NMS   Sec. II, paras. 3-4 (generalised)
 *   O10 coarse-to-fine refinement            Sec. II, para. 2 (top image first)
 *   O11 final selection                      Sec. II, para. 3
 *   O12 continuous (bilinear) score          extension beside Eq. (1)
 *   O13 similarity projection (scale)        Sec. II (other projection types
 *                                            than the rigid Eq. (2))
 *   O14 exhaustive (x, y, theta, scale)      as O8 over angles x scales
 *   O15 refinement at a chosen scale         as O10, scale kept
 *   O16 edge-taps-only vote (a reading)      Sec. II paras. 2-5 (the window)
 *   O17 gradient-map pyramid (a reading)     Sec. II, para. 2 (edge extraction
 *                                            followed by the pyramid)
 * Where the paper is silent the reading taken is stated at the function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ O1 */
/* Integer 3x3 Sobel on the interior; the one-pixel frame gets gx = gy = 0.
 * The paper names x- and y-gradients and magnitudes (Sec. II para. 2) but no
 * operator; the unnormalised integer Sobel pair is the reading taken. */
ORC_API void orc_sobel(const uint8_t* img, int W, int H, int32_t* gx, int32_t* gy)
{
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            size_t o = (size_t)y * W + x;
            if (x < 1 || y < 1 || x > W - 2 || y > H - 2) {
                gx[o] = 0;
                gy[o] = 0;
                continue;
            }
            int a = img[(size_t)(y - 1) * W + (x - 1)];
            int b = img[(size_t)(y - 1) * W + x];
            int c = img[(size_t)(y - 1) * W + (x + 1)];
            int d = img[(size_t)y * W + (x - 1)];
            int f = img[(size_t)y * W + (x + 1)];
            int g = img[(size_t)(y + 1) * W + (x - 1)];
            int h = img[(size_t)(y + 1) * W + x];
            int i = img[(size_t)(y + 1) * W + (x + 1)];
            gx[o] = (c + 2 * f + i) - (a + 2 * d + g);
            gy[o] = (g + 2 * h + i) - (a + 2 * b + c);
        }
    }
}

/* ------------------------------------------------------------------ O2 */
/* Squared threshold: a pixel is an edge iff gx^2 + gy^2 > floor(tau^2). */
ORC_API int64_t orc_edge_threshold(double tau)
{
    return (int64_t)floor(tau * tau);
}

/* Unit gradient direction at edge pixels, (0, 0) elsewhere.  g holds
 * (x, y) pairs, row-major.  Returns the number of edge pixels. */
ORC_API int orc_edge_field(const int32_t* gx, const int32_t* gy, int W, int H,
                           int64_t T2, double* g)
{
    int count = 0;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            size_t o = (size_t)y * W + x;
            int64_t m2 = (int64_t)gx[o] * gx[o] + (int64_t)gy[o] * gy[o];
            if (m2 > T2) {
                double m = sqrt((double)m2);
                g[2 * o + 0] = (double)gx[o] / m;
                g[2 * o + 1] = (double)gy[o] / m;
                ++count;
            } else {
                g[2 * o + 0] = 0.0;
                g[2 * o + 1] = 0.0;
            }
        }
    }
    return count;
}

/* ------------------------------------------------------------------ O3 */
/* One pyramid step: each output pixel is the rounded mean of a 2x2 block,
 * (sum + 2) >> 2; the output is floor(W/2) x floor(H/2). */
ORC_API void orc_pyr_down(const uint8_t* src, int W, int H, uint8_t* dst)
{
    int W2 = W / 2, H2 = H / 2;
    for (int y = 0; y < H2; ++y) {
        for (int x = 0; x < W2; ++x) {
            int s = src[(size_t)(2 * y) * W + 2 * x] + src[(size_t)(2 * y) * W + 2 * x + 1] +
                    src[(size_t)(2 * y + 1) * W + 2 * x] + src[(size_t)(2 * y + 1) * W + 2 * x + 1];
            dst[(size_t)y * W2 + x] = (uint8_t)((s + 2) >> 2);
        }
    }
}

/* ----------------------------------------------------------------- O17 */
/* The other reading of "edge extraction followed by an image pyramid"
 * (Sec. II para. 2): the Sobel gradients of the full image are extracted once
 * and the pyramid is built over the gradient maps, each component of level
 * l+1 being the floored mean floor((s + 2) / 4) of the 2x2 block sum s of
 * level l (the grey pyramid's rounding, on signed values); floor(W/2) x
 * floor(H/2).  Edges and directions then follow O2 on every level with the
 * same threshold. */
static int32_t orc_floor_div4(int32_t v)
{
    int32_t q = v / 4;          /* C division truncates toward zero */
    if (v % 4 != 0 && v < 0) q -= 1;
    return q;
}

ORC_API void orc_grad_down(const int32_t* gx, const int32_t* gy, int W, int H, int32_t* ox, int32_t* oy)
{
    int W2 = W / 2, H2 = H / 2;
    for (int y = 0; y < H2; ++y) {
        for (int x = 0; x < W2; ++x) {
            size_t a = (size_t)(2 * y) * W + 2 * x, b = a + W;
            int32_t sx = gx[a] + gx[a + 1] + gx[b] + gx[b + 1];
            int32_t sy = gy[a] + gy[a + 1] + gy[b] + gy[b + 1];
            ox[(size_t)y * W2 + x] = orc_floor_div4(sx + 2);
            oy[(size_t)y * W2 + x] = orc_floor_div4(sy + 2);
        }
    }
}

/* ------------------------------------------------------------------ O4 */
/* Model edge points of one level, row-major: t = (x - floor(W/2),
 * y - floor(H/2)) and the unit direction d.  Returns n, or -1 if more than
 * cap points exist. */
ORC_API int orc_model_points(const double* g, int W, int H, int32_t* t, double* d, int cap)
{
    int n = 0;
    int cx = W / 2, cy = H / 2;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            size_t o = (size_t)y * W + x;
            if (g[2 * o] == 0.0 && g[2 * o + 1] == 0.0) continue;
            if (n >= cap) return -1;
            t[2 * n + 0] = x - cx;
            t[2 * n + 1] = y - cy;
            d[2 * n + 0] = g[2 * o + 0];
            d[2 * n + 1] = g[2 * o + 1];
            ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------------ O5 */
/* Angle step at level l of an L-level pyramid: the top step halves at every
 * level going down (ldexp is an exact division by a power of two). */
ORC_API double orc_level_step(double step_top, int L, int l)
{
    return ldexp(step_top, -(L - 1 - l));
}

/* Number of angles at a level.  A full circle (range >= 360) wraps and does
 * not repeat 360; a partial range includes both end points (so a 90 degree
 * range at 3 degree steps has 31 angles). */
ORC_API int orc_level_count(double range, double step_l)
{
    if (range >= 360.0) return (int)ceil(360.0 / step_l);
    return (int)floor(range / step_l + 1e-9) + 1;
}

/* theta_k = theta_min + k * step, evaluated as a product then a sum. */
ORC_API double orc_theta(double theta_min, double step_l, int k)
{
    return theta_min + (double)k * step_l;
}

/* Wrap (full circle) or clamp (partial range) an angle index. */
ORC_API int orc_angle_index(int k, int K, int full)
{
    if (full) {
        int m = k % K;
        return m < 0 ? m + K : m;
    }
    return k < 0 ? 0 : (k > K - 1 ? K - 1 : k);
}

/* ------------------------------------------------------------------ O6 */
/* cos and sin of an angle in degrees, reduced exactly to one quadrant so that
 * multiples of 90 degrees give exact 0 and +-1. */
ORC_API void orc_sincos_deg(double deg, double* c, double* s)
{
    double r = fmod(deg, 360.0);
    if (r < 0.0) r += 360.0;
    if (r >= 360.0) r -= 360.0;
    int q = (int)floor(r / 90.0);
    if (q > 3) q = 3;
    double phi = r - 90.0 * (double)q;
    double rad = phi * (M_PI / 180.0);
    double c0 = cos(rad), s0 = sin(rad);
    switch (q) {
        case 0: *c = c0;  *s = s0;  break;
        case 1: *c = -s0; *s = c0;  break;
        case 2: *c = -c0; *s = -s0; break;
        default: *c = s0; *s = -c0; break;
    }
}

/* Eq. (2) without the translation: q_i is R(theta) t_i rounded half-up with a
 * 1e-9 snap (so that exact halves such as 3 sin 30 deg round up even when the
 * FP64 sine falls one ulp short), r_i = R(theta) d_i is the rotated model
 * direction used as p_i in Eq. (1). */
ORC_API void orc_rotate(int n, const int32_t* t, const double* d, double theta_deg,
                        int32_t* q, double* r)
{
    double c, s;
    orc_sincos_deg(theta_deg, &c, &s);
    for (int i = 0; i < n; ++i) {
        double tx = (double)t[2 * i], ty = (double)t[2 * i + 1];
        double vx = c * tx - s * ty;
        double vy = s * tx + c * ty;
        q[2 * i + 0] = (int32_t)floor(vx + 0.5 + 1e-9);
        q[2 * i + 1] = (int32_t)floor(vy + 0.5 + 1e-9);
        double dx = d[2 * i], dy = d[2 * i + 1];
        r[2 * i + 0] = c * dx - s * dy;
        r[2 * i + 1] = s * dx + c * dy;
    }
}

/* ------------------------------------------------------------------ O7 */
/* Eq. (1) with the per-point neighbouring search: every model point votes the
 * best cosine r_i . g over a win x win window centred on its projected
 * position u + q_i; pixels outside the image or off the edge set vote 0; the
 * sum is divided by the model's point count n (occluded points lower the
 * score, Sec. II para. 6).  S1 is the same sum with the centre tap only.
 *
 * O16, vote = 1: the other reading of the neighbouring search, in which only
 * edge pixels of the window take part.  A point's vote is the best cosine over
 * the edge pixels of its window, or 0 when the window holds none; pixels off
 * the edge set (field (0, 0)) and outside the image are skipped instead of
 * voting 0.  S1 is the same in both readings. */
ORC_API void orc_score(const double* g, int W, int H, int n, const int32_t* q, const double* r,
                       int ux, int uy, int win, int vote, double* Sw, double* S1)
{
    int h = (win - 1) / 2;
    double sw = 0.0, s1 = 0.0;
    for (int i = 0; i < n; ++i) {
        int px = ux + q[2 * i], py = uy + q[2 * i + 1];
        double rx = r[2 * i], ry = r[2 * i + 1];
        double best = -INFINITY;
        int edges = 0;
        for (int dy = -h; dy <= h; ++dy) {
            for (int dx = -h; dx <= h; ++dx) {
                int X = px + dx, Y = py + dy;
                double v = 0.0;
                int edge = 0;
                if (X >= 0 && X < W && Y >= 0 && Y < H) {
                    size_t o = (size_t)Y * W + X;
                    v = rx * g[2 * o] + ry * g[2 * o + 1];
                    edge = g[2 * o] != 0.0 || g[2 * o + 1] != 0.0;
                }
                if (vote == 1 && !edge) continue;
                edges += edge;
                if (v > best) best = v;
            }
        }
        if (vote == 1 && edges == 0) best = 0.0;
        double centre = 0.0;
        if (px >= 0 && px < W && py >= 0 && py < H) {
            size_t o = (size_t)py * W + px;
            centre = rx * g[2 * o] + ry * g[2 * o + 1];
        }
        sw += best;
        s1 += centre;
    }
    *Sw = sw / (double)n;
    *S1 = s1 / (double)n;
}

/* ------------------------------------------------------------------ O8 */
/* Exhaustive search at one level: every translation on the step grid
 * (x = i*sx < W, y = j*sy < H) and every angle k < K.  Per translation the
 * best angle is kept by the key (S_w desc, S_1 desc, k asc): angles are
 * visited in ascending order and replaced only by a strictly better score,
 * the "better score" rule of Sec. II para. 3.  Output maps are indexed
 * [j][i] with Gw = ceil(W/sx) columns.  Rows run in parallel when nthreads
 * > 1; every translation is independent, so the result does not depend on
 * it. */
ORC_API void orc_top_map(const double* g, int W, int H, int n, const int32_t* t, const double* d,
                         double theta_min, double step, int K, int sx, int sy, int win, int vote,
                         double* mapw, double* map1, int32_t* mapk, int nthreads)
{
    int Gw = (W + sx - 1) / sx, Gh = (H + sy - 1) / sy;
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n * K);
    double* r = (double*)malloc(sizeof(double) * 2 * (size_t)n * K);
    for (int k = 0; k < K; ++k)
        orc_rotate(n, t, d, orc_theta(theta_min, step, k), q + 2 * (size_t)n * k, r + 2 * (size_t)n * k);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int j = 0; j < Gh; ++j) {
        for (int i = 0; i < Gw; ++i) {
            double bw = -INFINITY, b1 = -INFINITY;
            int bk = -1;
            for (int k = 0; k < K; ++k) {
                double sw, s1;
                orc_score(g, W, H, n, q + 2 * (size_t)n * k, r + 2 * (size_t)n * k, i * sx, j * sy, win, vote,
                          &sw, &s1);
                if (sw > bw || (sw == bw && s1 > b1)) {
                    bw = sw;
                    b1 = s1;
                    bk = k;
                }
            }
            size_t o = (size_t)j * Gw + i;
            mapw[o] = bw;
            map1[o] = b1;
            mapk[o] = bk;
        }
    }
    free(q);
    free(r);
}

/* ------------------------------------------------------------- O9, O11 */
/* A candidate: pose (x, y, k) at a level and its two scores. */
typedef struct {
    double sw, s1;
    int32_t x, y, k;
} orc_cand;

/* Total order used for every selection: S_w desc, S_1 desc, x asc, y asc,
 * k asc.  The paper keeps the first pose found in x, y, theta loop order on a
 * tie of the score; S_1 is added ahead of position because the 3x3 vote makes
 * plateaus of equal S_w around a clean match. */
static int orc_better(const orc_cand* a, const orc_cand* b)
{
    if (a->sw != b->sw) return a->sw > b->sw;
    if (a->s1 != b->s1) return a->s1 > b->s1;
    if (a->x != b->x) return a->x < b->x;
    if (a->y != b->y) return a->y < b->y;
    return a->k < b->k;
}

static int orc_cmp(const void* pa, const void* pb)
{
    const orc_cand* a = (const orc_cand*)pa;
    const orc_cand* b = (const orc_cand*)pb;
    if (orc_better(a, b)) return -1;
    if (orc_better(b, a)) return 1;
    return 0;
}

/* Greedy non-maximum suppression over candidates sorted by the key: accept a
 * candidate iff its distance to every accepted one, scaled to level 0 by
 * 2^level, is >= dmin; stop after max_out.  Squared distances are compared
 * exactly: the integer part is exact in double and dmin is a float value, so
 * its square is exact too. */
static int orc_greedy_nms(const orc_cand* sorted, int n, int level, float dmin, int max_out,
                          orc_cand* out)
{
    double dmin2 = (double)dmin * (double)dmin;
    int m = 0;
    for (int c = 0; c < n && m < max_out; ++c) {
        int keep = 1;
        for (int a = 0; a < m; ++a) {
            int64_t dx = (int64_t)sorted[c].x - out[a].x;
            int64_t dy = (int64_t)sorted[c].y - out[a].y;
            int64_t d2 = (dx * dx + dy * dy) << (2 * level);
            if ((double)d2 < dmin2) {
                keep = 0;
                break;
            }
        }
        if (keep) out[m++] = sorted[c];
    }
    return m;
}

/* O9: a grid point is a candidate iff S_w >= min_score and its key (with the
 * position tie-break) is strictly better than that of each of its existing
 * 8 grid neighbours.  Candidates are sorted by the key and thinned by greedy
 * NMS.  Map layout as in orc_top_map.  Output arrays hold max_out entries;
 * returns the number written. */
ORC_API int orc_select(const double* mapw, const double* map1, const int32_t* mapk, int Gw, int Gh,
                       int sx, int sy, int level, double min_score, float dmin, int max_out,
                       int32_t* ox, int32_t* oy, int32_t* ok, double* ow, double* o1)
{
    orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * ((size_t)Gw * Gh + 1));
    int nc = 0;
    for (int j = 0; j < Gh; ++j) {
        for (int i = 0; i < Gw; ++i) {
            size_t o = (size_t)j * Gw + i;
            if (!(mapw[o] >= min_score)) continue;
            orc_cand me = {mapw[o], map1[o], i * sx, j * sy, mapk[o]};
            int is_max = 1;
            for (int b = -1; b <= 1 && is_max; ++b) {
                for (int a = -1; a <= 1; ++a) {
                    if (a == 0 && b == 0) continue;
                    int ii = i + a, jj = j + b;
                    if (ii < 0 || ii >= Gw || jj < 0 || jj >= Gh) continue;
                    size_t p = (size_t)jj * Gw + ii;
                    orc_cand nb = {mapw[p], map1[p], ii * sx, jj * sy, mapk[p]};
                    if (!orc_better(&me, &nb)) {
                        is_max = 0;
                        break;
                    }
                }
            }
            if (is_max) c[nc++] = me;
        }
    }
    qsort(c, (size_t)nc, sizeof(orc_cand), orc_cmp);
    orc_cand* out = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(max_out > 0 ? max_out : 1));
    int m = orc_greedy_nms(c, nc, level, dmin, max_out, out);
    for (int a = 0; a < m; ++a) {
        ox[a] = out[a].x;
        oy[a] = out[a].y;
        ok[a] = out[a].k;
        ow[a] = out[a].sw;
        o1[a] = out[a].s1;
    }
    free(out);
    free(c);
    return m;
}

/* ----------------------------------------------------------------- O10 */
/* One refinement step from level l+1 to level l for each candidate: the 27
 * poses (2x+a, 2y+b, 2k+c), a, b, c in {-1, 0, 1}, positions outside the
 * level image dropped, angle indices wrapped (full circle) or clamped; the
 * best by the key replaces the candidate.  g, W, H describe level l; t, d its
 * model points; step_l and K the level's angle grid. */
ORC_API void orc_refine_level(const double* g, int W, int H, int n, const int32_t* t, const double* d,
                              double theta_min, double step_l, int K, int full, int win, int vote, int nc,
                              int32_t* cx, int32_t* cy, int32_t* ck, double* cw, double* c1)
{
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n);
    double* r = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    for (int c = 0; c < nc; ++c) {
        orc_cand best = {-INFINITY, -INFINITY, 0, 0, 0};
        int have = 0;
        for (int dk = -1; dk <= 1; ++dk) {
            int k = orc_angle_index(2 * ck[c] + dk, K, full);
            orc_rotate(n, t, d, orc_theta(theta_min, step_l, k), q, r);
            for (int b = -1; b <= 1; ++b) {
                for (int a = -1; a <= 1; ++a) {
                    int x = 2 * cx[c] + a, y = 2 * cy[c] + b;
                    if (x < 0 || x >= W || y < 0 || y >= H) continue;
                    orc_cand me;
                    orc_score(g, W, H, n, q, r, x, y, win, vote, &me.sw, &me.s1);
                    me.x = x;
                    me.y = y;
                    me.k = k;
                    if (!have || orc_better(&me, &best)) {
                        best = me;
                        have = 1;
                    }
                }
            }
        }
        cx[c] = best.x;
        cy[c] = best.y;
        ck[c] = best.k;
        cw[c] = best.sw;
        c1[c] = best.s1;
    }
    free(q);
    free(r);
}

/* ----------------------------------------------------------------- O11 */
/* Final selection at level 0: sort by the key, greedy NMS, keep S_w >=
 * min_score, at most max_out.  Arrays are in/out: the first m entries on
 * return are the result. */
ORC_API int orc_final(int nc, int32_t* cx, int32_t* cy, int32_t* ck, double* cw, double* c1,
                      double min_score, float dmin, int max_out)
{
    orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(nc > 0 ? nc : 1));
    int m0 = 0;
    for (int a = 0; a < nc; ++a) {
        if (!(cw[a] >= min_score)) continue;
        orc_cand e = {cw[a], c1[a], cx[a], cy[a], ck[a]};
        c[m0++] = e;
    }
    qsort(c, (size_t)m0, sizeof(orc_cand), orc_cmp);
    orc_cand* out = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(max_out > 0 ? max_out : 1));
    int m = orc_greedy_nms(c, m0, 0, dmin, max_out, out);
    for (int a = 0; a < m; ++a) {
        cx[a] = out[a].x;
        cy[a] = out[a].y;
        ck[a] = out[a].k;
        cw[a] = out[a].sw;
        c1[a] = out[a].s1;
    }
    free(out);
    free(c);
    return m;
}

/* ----------------------------------------------------------------- O12 */
/* Continuous score (an extension beside Eq. (1)): the mean over the model's
 * points of r_i . B(R(theta) t_i + u), B the bilinear interpolation of the
 * unit-direction field (0 off the edge set and outside the image), with no
 * window and no rounding of positions; theta in degrees.  Also its gradient
 * with respect to (u_x, u_y, theta_deg): per point,
 *   d/du   = J_B(p)^T r,
 *   d/dth  = (pi/180) [ (R' d) . B(p) + r . (J_B(p) R' t) ],
 * R' = dR/dtheta_rad, J_B the 2x2 Jacobian of B in the cell containing p
 * (cells are [x0, x0+1) x [y0, y0+1), x0 = floor(p_x)). */
static void orc_field_at(const double* g, int W, int H, int x, int y, double* vx, double* vy)
{
    if (x < 0 || x >= W || y < 0 || y >= H) {
        *vx = 0.0;
        *vy = 0.0;
        return;
    }
    size_t o = (size_t)y * W + x;
    *vx = g[2 * o];
    *vy = g[2 * o + 1];
}

ORC_API void orc_cont_score(const double* g, int W, int H, int n, const int32_t* t, const double* d,
                            double ux, double uy, double theta_deg, double* S, double* grad)
{
    double c, s;
    orc_sincos_deg(theta_deg, &c, &s);
    const double k = M_PI / 180.0;
    double sum = 0.0, gx = 0.0, gy = 0.0, gt = 0.0;
    for (int i = 0; i < n; ++i) {
        double tx = (double)t[2 * i], ty = (double)t[2 * i + 1];
        double dx = d[2 * i], dy = d[2 * i + 1];
        double px = c * tx - s * ty + ux;
        double py = s * tx + c * ty + uy;
        double rx = c * dx - s * dy, ry = s * dx + c * dy;
        double x0 = floor(px), y0 = floor(py);
        double fx = px - x0, fy = py - y0;
        int ix = (int)x0, iy = (int)y0;
        double a00x, a00y, a10x, a10y, a01x, a01y, a11x, a11y;
        orc_field_at(g, W, H, ix, iy, &a00x, &a00y);
        orc_field_at(g, W, H, ix + 1, iy, &a10x, &a10y);
        orc_field_at(g, W, H, ix, iy + 1, &a01x, &a01y);
        orc_field_at(g, W, H, ix + 1, iy + 1, &a11x, &a11y);
        double bx = (1 - fx) * (1 - fy) * a00x + fx * (1 - fy) * a10x + (1 - fx) * fy * a01x + fx * fy * a11x;
        double by = (1 - fx) * (1 - fy) * a00y + fx * (1 - fy) * a10y + (1 - fx) * fy * a01y + fx * fy * a11y;
        /* Jacobian columns: dB/dpx, dB/dpy */
        double bxx = (1 - fy) * (a10x - a00x) + fy * (a11x - a01x);
        double byx = (1 - fy) * (a10y - a00y) + fy * (a11y - a01y);
        double bxy = (1 - fx) * (a01x - a00x) + fx * (a11x - a10x);
        double byy = (1 - fx) * (a01y - a00y) + fx * (a11y - a10y);
        double v = rx * bx + ry * by;
        double dpx = rx * bxx + ry * byx; /* r . dB/dpx */
        double dpy = rx * bxy + ry * byy; /* r . dB/dpy */
        /* R' t and R' d (derivative with respect to theta in radians) */
        double rtx = -s * tx - c * ty, rty = c * tx - s * ty;
        double rdx = -s * dx - c * dy, rdy = c * dx - s * dy;
        sum += v;
        gx += dpx;
        gy += dpy;
        gt += (rdx * bx + rdy * by) + (rtx * dpx + rty * dpy);
    }
    *S = sum / (double)n;
    grad[0] = gx / (double)n;
    grad[1] = gy / (double)n;
    grad[2] = k * gt / (double)n;
}

/* ----------------------------------------------------------------- O13 */
/* The paper names other projection types than its rigid Eq. (2); this is the
 * similarity pose: p_i = sigma R(theta) t_i + u.  q_i rounds sigma times the
 * rotated offset (rotation first, as in O6, then the product with sigma) with
 * the same half-up rule and 1e-9 snap; r_i = R(theta) d_i, since a uniform
 * scale leaves directions unchanged.  sigma = 1 gives O6 exactly. */
ORC_API void orc_project(int n, const int32_t* t, const double* d, double theta_deg, double sigma,
                         int32_t* q, double* r)
{
    double c, s;
    orc_sincos_deg(theta_deg, &c, &s);
    for (int i = 0; i < n; ++i) {
        double tx = (double)t[2 * i], ty = (double)t[2 * i + 1];
        double vx = c * tx - s * ty;
        double vy = s * tx + c * ty;
        vx = sigma * vx;
        vy = sigma * vy;
        q[2 * i + 0] = (int32_t)floor(vx + 0.5 + 1e-9);
        q[2 * i + 1] = (int32_t)floor(vy + 0.5 + 1e-9);
        double dx = d[2 * i], dy = d[2 * i + 1];
        r[2 * i + 0] = c * dx - s * dy;
        r[2 * i + 1] = s * dx + c * dy;
    }
}

/* Scale j of the grid sigma_min + j * sigma_step (a product, not a running
 * sum). */
ORC_API double orc_scale(double sigma_min, double sigma_step, int j)
{
    return sigma_min + (double)j * sigma_step;
}

/* ----------------------------------------------------------------- O14 */
/* O8 over angles and scales: every translation on the step grid, every angle
 * k < K and scale j < S; the pose index is m = j K + k (scale-major), and per
 * translation the best m is kept by the key (S_w desc, S_1 desc, m asc):
 * indices visited in ascending order, replaced only by a strictly better
 * score.  With S = 1 and sigma 1 this is O8. */
ORC_API void orc_top_map_sim(const double* g, int W, int H, int n, const int32_t* t, const double* d,
                             double theta_min, double step, int K, double sigma_min, double sigma_step, int S,
                             int sx, int sy, int win, int vote, double* mapw, double* map1, int32_t* mapk,
                             int nthreads)
{
    int Gw = (W + sx - 1) / sx, Gh = (H + sy - 1) / sy;
    int M = K * S;
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n * M);
    double* r = (double*)malloc(sizeof(double) * 2 * (size_t)n * M);
    for (int j = 0; j < S; ++j)
        for (int k = 0; k < K; ++k) {
            int m = j * K + k;
            orc_project(n, t, d, orc_theta(theta_min, step, k), orc_scale(sigma_min, sigma_step, j),
                        q + 2 * (size_t)n * m, r + 2 * (size_t)n * m);
        }
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int y = 0; y < Gh; ++y) {
        for (int x = 0; x < Gw; ++x) {
            double bw = -INFINITY, b1 = -INFINITY;
            int bm = -1;
            for (int m = 0; m < M; ++m) {
                double sw, s1;
                orc_score(g, W, H, n, q + 2 * (size_t)n * m, r + 2 * (size_t)n * m, x * sx, y * sy, win, vote,
                          &sw, &s1);
                if (sw > bw || (sw == bw && s1 > b1)) {
                    bw = sw;
                    b1 = s1;
                    bm = m;
                }
            }
            size_t o = (size_t)y * Gw + x;
            mapw[o] = bw;
            map1[o] = b1;
            mapk[o] = bm;
        }
    }
    free(q);
    free(r);
}

/* ----------------------------------------------------------------- O15 */
/* O10 at the candidate's scale: a candidate of level l+1 carries the pose
 * index m = j K_above + k; at level l the 27 poses (2x+a, 2y+b, 2k+c) are
 * scored at scale j (the scale grid is the same on every level, so there is
 * nothing finer to refine) and the best by the key (S_w, S_1, x, y, then the
 * level-l index j K + k') replaces the candidate, written back as that index.
 * With one scale this is O10. */
ORC_API void orc_refine_level_sim(const double* g, int W, int H, int n, const int32_t* t, const double* d,
                                  double theta_min, double step_l, int K, int K_above, int full, int win,
                                  int vote, double sigma_min, double sigma_step, int nc, int32_t* cx, int32_t* cy, int32_t* cm,
                                  double* cw, double* c1)
{
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)n);
    double* r = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    for (int c = 0; c < nc; ++c) {
        int j = cm[c] / K_above, k0 = cm[c] % K_above;
        double sigma = orc_scale(sigma_min, sigma_step, j);
        orc_cand best = {-INFINITY, -INFINITY, 0, 0, 0};
        int have = 0;
        for (int dk = -1; dk <= 1; ++dk) {
            int k = orc_angle_index(2 * k0 + dk, K, full);
            orc_project(n, t, d, orc_theta(theta_min, step_l, k), sigma, q, r);
            for (int b = -1; b <= 1; ++b) {
                for (int a = -1; a <= 1; ++a) {
                    int x = 2 * cx[c] + a, y = 2 * cy[c] + b;
                    if (x < 0 || x >= W || y < 0 || y >= H) continue;
                    orc_cand me;
                    orc_score(g, W, H, n, q, r, x, y, win, vote, &me.sw, &me.s1);
                    me.x = x;
                    me.y = y;
                    me.k = j * K + k;
                    if (!have || orc_better(&me, &best)) {
                        best = me;
                        have = 1;
                    }
                }
            }
        }
        cx[c] = best.x;
        cy[c] = best.y;
        cm[c] = best.k;
        cw[c] = best.sw;
        c1[c] = best.s1;
    }
    free(q);
    free(r);
}
