// Coarse-to-fine refinement.  The paper starts the score computation at the
// top image of the pyramid (Sec. II para. 2); each candidate found there is
// carried down one level at a time by re-scoring the 27 poses
// (2x + a, 2y + b, 2k + c), a, b, c in {-1, 0, 1}, with the same windowed
// score (Eq. 1) and keeping the best by the selection key.
//
// One workgroup per candidate, 3 groups of 5 waves, one group per angle
// 2k - 1, 2k, 2k + 1.  A thread takes model points i = j, j + 320, ...; for
// each it forms q_i and r_i in FP64, reads the 5x5 field block that covers
// the 3x3 windows of all 9 translations, and accumulates 9 windowed votes and
// 9 centre votes.  Partial sums are combined by a fixed butterfly per wave
// and in wave order across the group, so results are deterministic.
#include "tm_device.h"

namespace tmk {

namespace {

constexpr int kGroup = 320;         // threads per angle group (5 waves)
constexpr int kWaves = kGroup / 64;

__global__ __launch_bounds__(960) void k_refine(RefineArgs a, tm_pose* __restrict__ poses, int n,
                                                 const int32_t* __restrict__ n_dev)
{
    __shared__ float red_w[3][kWaves][9], red_1[3][kWaves][9];
    __shared__ int cur_x, cur_y, cur_k;
    __shared__ float cur_w, cur_1;
    const int c = blockIdx.x;
    int count = n;
    if (n_dev) count = min(count, *n_dev);
    if (c >= count) return;

    const int grp = threadIdx.x / kGroup, j = threadIdx.x - grp * kGroup;
    const int wv = j >> 6, lane = threadIdx.x & 63;
    const tm_pose p0 = poses[c];
    int x = p0.x, y = p0.y, k = p0.k;
    float bw = p0.score_w, b1 = p0.score_1;
    const int h = 1;  // the 27-pose neighbourhood is +-1 at every level

    for (int l = min(p0.level, a.L - 1) - 1; l >= 0; --l) {
        const RefineLevel L = a.lv[l];
        const int kc = angle_index(2 * k + grp - 1, L.K, a.full);
        double cs, sn;
        sincos_deg(level_theta(a.theta_min, L.step, kc), &cs, &sn);
        float aw[9], a1[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) {
            aw[m] = 0.f;
            a1[m] = 0.f;
        }
        const int wh = (a.win - 1) / 2;
        for (int i = j; i < L.n; i += kGroup) {
            int qx, qy;
            double rx, ry;
            project_point(L.pts[i], cs, sn, &qx, &qy, &rx, &ry);
            const float fx = (float)rx, fy = (float)ry;
            const int px = 2 * x + qx, py = 2 * y + qy;
            if (wh == 1) {
                float D[5][5];
#pragma unroll
                for (int v = 0; v < 5; ++v)
#pragma unroll
                    for (int u = 0; u < 5; ++u)
                        D[v][u] = field_dot(L.field, a.precision, L.W, L.H, px - 2 + u, py - 2 + v, fx, fy);
                float hm[5][3];
#pragma unroll
                for (int v = 0; v < 5; ++v)
#pragma unroll
                    for (int u = 0; u < 3; ++u) hm[v][u] = fmaxf(fmaxf(D[v][u], D[v][u + 1]), D[v][u + 2]);
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        aw[b * 3 + u] += fmaxf(fmaxf(hm[b][u], hm[b + 1][u]), hm[b + 2][u]);
                        a1[b * 3 + u] += D[b + 1][u + 1];
                    }
            } else {
                // any odd window: direct evaluation of each translation
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        const int cx = px + u - h, cy = py + b - h;
                        float best = -INFINITY;
                        for (int dy = -wh; dy <= wh; ++dy)
                            for (int dx = -wh; dx <= wh; ++dx)
                                best = fmaxf(best, field_dot(L.field, a.precision, L.W, L.H, cx + dx, cy + dy, fx, fy));
                        aw[b * 3 + u] += best;
                        a1[b * 3 + u] += field_dot(L.field, a.precision, L.W, L.H, cx, cy, fx, fy);
                    }
            }
        }
#pragma unroll
        for (int m = 0; m < 9; ++m) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                aw[m] += __shfl_xor(aw[m], off, 64);
                a1[m] += __shfl_xor(a1[m], off, 64);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int m = 0; m < 9; ++m) {
                red_w[grp][wv][m] = aw[m];
                red_1[grp][wv][m] = a1[m];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const float nf = (float)L.n;
            bool have = false;
            int bx = 0, by = 0, bkk = 0;
            for (int g = 0; g < 3; ++g) {
                const int kg = angle_index(2 * k + g - 1, L.K, a.full);
                for (int b = 0; b < 3; ++b)
                    for (int u = 0; u < 3; ++u) {
                        const int xx = 2 * x + u - 1, yy = 2 * y + b - 1;
                        if (xx < 0 || yy < 0 || xx >= L.W || yy >= L.H) continue;
                        float sw = 0.f, s1 = 0.f;
                        for (int w = 0; w < kWaves; ++w) {
                            sw += red_w[g][w][b * 3 + u];
                            s1 += red_1[g][w][b * 3 + u];
                        }
                        sw /= nf;
                        s1 /= nf;
                        if (!have || key_better(sw, s1, xx, yy, kg, bw, b1, bx, by, bkk)) {
                            have = true;
                            bw = sw;
                            b1 = s1;
                            bx = xx;
                            by = yy;
                            bkk = kg;
                        }
                    }
            }
            cur_x = bx;
            cur_y = by;
            cur_k = bkk;
            cur_w = bw;
            cur_1 = b1;
        }
        __syncthreads();
        x = cur_x;
        y = cur_y;
        k = cur_k;
        bw = cur_w;
        b1 = cur_1;
    }
    if (threadIdx.x == 0) {
        tm_pose o;
        o.x = x;
        o.y = y;
        o.k = k;
        o.level = 0;
        o.theta_deg = (float)level_theta(a.theta_min, a.lv[0].step, k);
        o.score_w = bw;
        o.score_1 = b1;
        o.reserved = 0;
        poses[c] = o;
    }
}

}  // namespace

hipError_t launch_refine(const RefineArgs& a, tm_pose* poses, int n, const int32_t* n_dev, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine, dim3(n), dim3(3 * kGroup), 0, s, a, poses, n, n_dev);
    return hipGetLastError();
}

}  // namespace tmk
