/*
 * Driver for a sanitizer build of the CPU oracle (test infrastructure): every
 * exported oracle routine is called on small seeded inputs, including poses
 * whose windows leave the image, partial angle ranges, both window votes,
 * scaled projections, empty candidate lists and the continuous score at the
 * image border.  Built with -fsanitize=address,undefined by
 * tests/test_oracle_sanitize.py and run as a child process; any out-of-bounds
 * access, leak or undefined operation ends it with a report.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_sobel(const uint8_t* img, int W, int H, int32_t* gx, int32_t* gy);
int64_t orc_edge_threshold(double tau);
int orc_edge_field(const int32_t* gx, const int32_t* gy, int W, int H, int64_t T2, double* g);
void orc_pyr_down(const uint8_t* src, int W, int H, uint8_t* dst);
void orc_grad_down(const int32_t* gx, const int32_t* gy, int W, int H, int32_t* ox, int32_t* oy);
int orc_model_points(const double* g, int W, int H, int32_t* t, double* d, int cap);
double orc_level_step(double step_top, int L, int l);
int orc_level_count(double range, double step_l);
double orc_theta(double theta_min, double step_l, int k);
int orc_angle_index(int k, int K, int full);
void orc_sincos_deg(double deg, double* c, double* s);
void orc_rotate(int n, const int32_t* t, const double* d, double theta_deg, int32_t* q, double* r);
void orc_score(const double* g, int W, int H, int n, const int32_t* q, const double* r, int ux, int uy, int win,
               int vote, double* Sw, double* S1);
void orc_top_map(const double* g, int W, int H, int n, const int32_t* t, const double* d, double theta_min,
                 double step, int K, int sx, int sy, int win, int vote, double* mapw, double* map1, int32_t* mapk,
                 int nthreads);
int orc_select(const double* mapw, const double* map1, const int32_t* mapk, int Gw, int Gh, int sx, int sy, int level,
               double min_score, float dmin, int max_out, int32_t* ox, int32_t* oy, int32_t* ok, double* ow,
               double* o1);
void orc_refine_level(const double* g, int W, int H, int n, const int32_t* t, const double* d, double theta_min,
                      double step_l, int K, int full, int win, int vote, int nc, int32_t* cx, int32_t* cy,
                      int32_t* ck, double* cw, double* c1);
int orc_final(int nc, int32_t* cx, int32_t* cy, int32_t* ck, double* cw, double* c1, double min_score, float dmin,
              int max_out);
void orc_cont_score(const double* g, int W, int H, int n, const int32_t* t, const double* d, double ux, double uy,
                    double theta_deg, double* S, double* grad);
void orc_project(int n, const int32_t* t, const double* d, double theta_deg, double sigma, int32_t* q, double* r);
double orc_scale(double sigma_min, double sigma_step, int j);
void orc_top_map_sim(const double* g, int W, int H, int n, const int32_t* t, const double* d, double theta_min,
                     double step, int K, double sigma_min, double sigma_step, int S, int sx, int sy, int win,
                     int vote, double* mapw, double* map1, int32_t* mapk, int nthreads);
void orc_refine_level_sim(const double* g, int W, int H, int n, const int32_t* t, const double* d, double theta_min,
                          double step_l, int K, int K_above, int full, int win, int vote, double sigma_min,
                          double sigma_step, int nc, int32_t* cx, int32_t* cy, int32_t* cm, double* cw, double* c1);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 11);
}

#define W 41
#define H 37
#define MW 13
#define MH 12

int main(void)
{
    double sum = 0.0;
    uint8_t img[W * H], mimg[MW * MH], half[(W / 2) * (H / 2)], mhalf[(MW / 2) * (MH / 2)];
    for (int i = 0; i < W * H; ++i) img[i] = (uint8_t)(next_u32() & 255);
    for (int y = 0; y < MH; ++y)
        for (int x = 0; x < MW; ++x) mimg[y * MW + x] = (x >= 3 && x < 9 && y >= 2 && y < 8) ? 210 : 40;
    int32_t gx[W * H], gy[W * H], mgx[MW * MH], mgy[MW * MH];
    orc_sobel(img, W, H, gx, gy);
    orc_sobel(mimg, MW, MH, mgx, mgy);
    double* g = malloc(sizeof(double) * 2 * W * H);
    double* mg = malloc(sizeof(double) * 2 * MW * MH);
    const int64_t T2 = orc_edge_threshold(50.0);
    sum += orc_edge_field(gx, gy, W, H, T2, g);
    sum += orc_edge_field(mgx, mgy, MW, MH, orc_edge_threshold(30.0), mg);
    orc_pyr_down(img, W, H, half);
    orc_pyr_down(mimg, MW, MH, mhalf);
    int32_t ox[(W / 2) * (H / 2)], oy[(W / 2) * (H / 2)];
    orc_grad_down(gx, gy, W, H, ox, oy);
    for (int i = 0; i < (W / 2) * (H / 2); ++i) sum += half[i] + ox[i] + oy[i];
    int32_t t[MW * MH * 2];
    double d[MW * MH * 2];
    const int n = orc_model_points(mg, MW, MH, t, d, MW * MH);
    sum += n;
    double c, s;
    for (double a = -725.0; a <= 725.0; a += 37.5) {
        orc_sincos_deg(a, &c, &s);
        sum += c + s;
    }
    for (int L = 1; L <= 4; ++L)
        for (int l = 0; l < L; ++l) {
            const double st = orc_level_step(8.0, L, l);
            sum += orc_level_count(360.0, st) + orc_level_count(90.0, st) + orc_theta(-10.0, st, 3);
        }
    for (int k = -5; k < 80; k += 7) sum += orc_angle_index(k, 72, 1) + orc_angle_index(k, 31, 0);
    int32_t q[MW * MH * 2];
    double r[MW * MH * 2];
    orc_rotate(n, t, d, 33.0, q, r);
    orc_project(n, t, d, 210.0, 1.35, q, r);
    double Sw, S1;
    const int pos[6][2] = {{0, 0}, {W - 1, H - 1}, {-4, 3}, {W + 3, H / 2}, {20, 18}, {5, H - 2}};
    for (int p = 0; p < 6; ++p)
        for (int win = 1; win <= 5; win += 2)
            for (int vote = 0; vote <= 1; ++vote) {
                orc_rotate(n, t, d, 15.0 * p, q, r);
                orc_score(g, W, H, n, q, r, pos[p][0], pos[p][1], win, vote, &Sw, &S1);
                sum += Sw + S1;
            }
    const int K = 24, sx = 2, sy = 3, Gw = (W + sx - 1) / sx, Gh = (H + sy - 1) / sy;
    /* maps sized for the unit-step grid, the largest searched below */
    double* mw = malloc(sizeof(double) * W * H);
    double* m1 = malloc(sizeof(double) * W * H);
    int32_t* mk = malloc(sizeof(int32_t) * W * H);
    orc_top_map(g, W, H, n, t, d, 0.0, 15.0, K, sx, sy, 3, 0, mw, m1, mk, 2);
    int32_t cx[64], cy[64], ck[64];
    double cw[64], c1[64];
    int nc = orc_select(mw, m1, mk, Gw, Gh, sx, sy, 1, 0.05, 2.0f, 16, cx, cy, ck, cw, c1);
    sum += nc;
    sum += orc_select(mw, m1, mk, Gw, Gh, sx, sy, 0, 2.0, 2.0f, 16, cx, cy, ck, cw, c1);  /* none above the floor */
    orc_top_map(g, W, H, n, t, d, 0.0, 15.0, K, 1, 1, 5, 1, mw, m1, mk, 1);
    nc = orc_select(mw, m1, mk, W, H, 1, 1, 0, -1.0, 0.0f, 64, cx, cy, ck, cw, c1);
    orc_refine_level(g, W, H, n, t, d, 0.0, 7.5, 2 * K, 1, 3, 0, nc, cx, cy, ck, cw, c1);
    orc_refine_level(g, W, H, n, t, d, 0.0, 3.0, 31, 0, 3, 1, nc, cx, cy, ck, cw, c1);
    sum += orc_final(nc, cx, cy, ck, cw, c1, 0.0, 3.0f, 8);
    sum += orc_final(0, cx, cy, ck, cw, c1, 0.0, 3.0f, 8);
    orc_top_map_sim(g, W, H, n, t, d, 0.0, 30.0, 12, 0.8, 0.2, 3, 1, 1, 3, 0, mw, m1, mk, 2);
    for (int i = 0; i < 4; ++i) {
        cx[i] = 2 + 5 * i;
        cy[i] = 1 + 4 * i;
        ck[i] = (i % 3) * 12 + 5 * i;
    }
    orc_refine_level_sim(g, W, H, n, t, d, 0.0, 15.0, 24, 12, 1, 3, 1, 0.8, 0.2, 4, cx, cy, ck, cw, c1);
    sum += orc_scale(0.8, 0.2, 2);
    double S, grad[3];
    const double cpos[4][3] = {{0.0, 0.0, 10.0}, {W - 1.0, H - 1.0, 350.0}, {20.25, 17.75, 123.4}, {-3.5, 2.0, 0.0}};
    for (int p = 0; p < 4; ++p) {
        orc_cont_score(g, W, H, n, t, d, cpos[p][0], cpos[p][1], cpos[p][2], &S, grad);
        sum += S + grad[0] + grad[1] + grad[2];
    }
    for (int i = 0; i < W * H; ++i) sum += mw[i] + m1[i] + mk[i];
    free(mw);
    free(m1);
    free(mk);
    free(g);
    free(mg);
    printf("ok %.17g\n", sum);
    return isfinite(sum) ? 0 : 1;
}
