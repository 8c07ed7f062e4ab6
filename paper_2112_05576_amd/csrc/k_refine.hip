// Coarse-to-fine refinement.  The paper starts the score computation at the
// top image of the pyramid (Sec. II para. 2); each candidate found there is
// carried down one level at a time by re-scoring the 27 poses
// (2x + a, 2y + b, 2k + c), a, b, c in {-1, 0, 1}, with the same windowed
// score (Eq. 1) and keeping the best by the selection key.
//
// One launch per level.  The grid is (candidate x angle c x chunk of model
// points, pair), so that a level spreads over hundreds of workgroups.  A
// workgroup first picks its candidate's pose at the level above from that
// level's partial sums (every workgroup of the candidate makes the same pick,
// in the same order), then forms q_i and r_i of its points in FP64, reads the
// 5x5 field block covering the 3x3 windows of the 9 translations with all 25
// loads in flight, and accumulates 9 windowed votes and 9 centre votes.  Sums
// are combined by a fixed butterfly per wave and in wave order across the
// workgroup, then across chunks in chunk order at the pick.
#include "tm_device.h"

namespace tmk {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Best of the 27 poses around (x, y, k) (a pose of level l+1) at level l, from
// the partial sums part[g][chunk][m] (m < 9: S_w of translation m, m >= 9:
// S_1).  Runs on one wave; every lane returns the result.
__device__ void pick27(const float* __restrict__ part, int chunks, int x, int y, int k, int W, int H, int n, int K,
                       int full, float* bw, float* b1, int* bx, int* by, int* bk)
{
    const int lane = threadIdx.x & 63;
    const int m = lane < 27 ? lane : 26;
    const int g = m / 9, t = m % 9, b = t / 3, u = t % 3;
    const int kg = angle_index(2 * k + g - 1, K, full);
    const int xx = 2 * x + u - 1, yy = 2 * y + b - 1;
    float sw = 0.f, s1 = 0.f;
    for (int ch = 0; ch < chunks; ++ch) {
        const float* p = part + ((size_t)g * chunks + ch) * 18;
        sw += p[t];
        s1 += p[9 + t];
    }
    sw /= (float)n;
    s1 /= (float)n;
    const bool ok = lane < 27 && xx >= 0 && yy >= 0 && xx < W && yy < H;
    float kw = ok ? sw : -INFINITY, k1 = ok ? s1 : -INFINITY;
    int kx = ok ? xx : 0x7fffffff, ky = ok ? yy : 0x7fffffff, kk = ok ? kg : 0x7fffffff;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float ow = __shfl_xor(kw, off, 64), o1 = __shfl_xor(k1, off, 64);
        const int ox = __shfl_xor(kx, off, 64), oy = __shfl_xor(ky, off, 64), okk = __shfl_xor(kk, off, 64);
        if (key_better(ow, o1, ox, oy, okk, kw, k1, kx, ky, kk)) {
            kw = ow;
            k1 = o1;
            kx = ox;
            ky = oy;
            kk = okk;
        }
    }
    *bw = kw;
    *b1 = k1;
    *bx = kx;
    *by = ky;
    *bk = kk;
}

__device__ __forceinline__ int chunks_of(int n) { return (n + kThreads - 1) / kThreads; }

struct LevelArgs {
    int level;             // l, the level scored
    int max_chunks;        // largest chunk count of level l over the pairs (grid stride)
    int pick;              // 1: pick the pose of level l+1 from its partials; 0: poses are given
    int K, K_above;        // angles of levels l and l+1
    double step, step_above;
    int full, win, max_cand;
    double theta_min;
    int src;               // centre buffer read (0/1); the other one is written
};

template <int PREC>
__global__ __launch_bounds__(kThreads) void k_refine_level(LevelArgs a, const PairDesc* __restrict__ pairs)
{
    __shared__ float red[kWaves][18];
    __shared__ int cur[3];
    const PairDesc& P = pairs[blockIdx.y];
    const int l = a.level;
    const int chunks = chunks_of(P.n[l]);
    const int chunk = blockIdx.x % a.max_chunks;
    const int g = (blockIdx.x / a.max_chunks) % 3;
    const int c = blockIdx.x / (a.max_chunks * 3);
    if (chunk >= chunks) return;
    int count = a.max_cand;
    if (P.ncand) count = min(count, *P.ncand);
    if (c >= count) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    if (threadIdx.x < 64) {
        int x, y, k;
        float sw, s1;
        if (a.pick) {
            const tm_pose ctr = P.ctr[a.src][c];
            const int la = l + 1;
            pick27(P.part[la] + (size_t)c * 3 * chunks_of(P.n[la]) * 18, chunks_of(P.n[la]), ctr.x, ctr.y, ctr.k,
                   P.W[la], P.H[la], P.n[la], a.K_above, a.full, &sw, &s1, &x, &y, &k);
        } else {
            const tm_pose p = P.cand[c];
            x = p.x;
            y = p.y;
            k = p.k;
            sw = p.score_w;
            s1 = p.score_1;
        }
        if (lane == 0) {
            cur[0] = x;
            cur[1] = y;
            cur[2] = k;
            if (g == 0 && chunk == 0) {
                tm_pose o;
                o.x = x;
                o.y = y;
                o.k = k;
                o.level = l + 1;
                o.theta_deg = (float)level_theta(a.theta_min, a.step_above, k);
                o.score_w = sw;
                o.score_1 = s1;
                o.reserved = 0;
                P.ctr[a.src ^ 1][c] = o;
            }
        }
    }
    __syncthreads();
    const int x = cur[0], y = cur[1], k = cur[2];
    const void* field = P.field[l];
    const int W = P.W[l], H = P.H[l], n = P.n[l];
    const ModelPoint* __restrict__ pts = P.pts[l];
    const int kc = angle_index(2 * k + g - 1, a.K, a.full);
    double cs, sn;
    sincos_deg(level_theta(a.theta_min, a.step, kc), &cs, &sn);
    float aw[9], a1[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        aw[m] = 0.f;
        a1[m] = 0.f;
    }
    const int per = (n + chunks - 1) / chunks;
    const int i0 = chunk * per, i1 = min(n, i0 + per);
    const int wh = (a.win - 1) / 2;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += kThreads) {
        int qx, qy;
        double rx, ry;
        project_point(pts[i], cs, sn, &qx, &qy, &rx, &ry);
        const float fx = (float)rx, fy = (float)ry;
        const int px = 2 * x + qx, py = 2 * y + qy;
        if (wh == 1) {
            // the 5x5 block covering the 3x3 windows of the 9 translations:
            // all 25 loads are issued before any is used
            int col[5];
            size_t rowoff[5];
            bool cin[5], rin[5];
#pragma unroll
            for (int u = 0; u < 5; ++u) {
                const int xx = px - 2 + u, yy = py - 2 + u;
                cin[u] = (unsigned)xx < (unsigned)W;
                rin[u] = (unsigned)yy < (unsigned)H;
                col[u] = min(max(xx, 0), W - 1);
                rowoff[u] = (size_t)min(max(yy, 0), H - 1) * W;
            }
            float2 gv[5][5];
#pragma unroll
            for (int v = 0; v < 5; ++v)
#pragma unroll
                for (int u = 0; u < 5; ++u) gv[v][u] = field_load<PREC>(field, rowoff[v] + col[u]);
            __builtin_amdgcn_sched_barrier(0);
            float D[5][5];
#pragma unroll
            for (int v = 0; v < 5; ++v)
#pragma unroll
                for (int u = 0; u < 5; ++u) {
                    const float d = fx * gv[v][u].x + fy * gv[v][u].y;
                    D[v][u] = (rin[v] && cin[u]) ? d : 0.0f;
                }
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
                    const int cx = px + u - 1, cy = py + b - 1;
                    float best = -INFINITY;
                    for (int dy = -wh; dy <= wh; ++dy)
                        for (int dx = -wh; dx <= wh; ++dx)
                            best = fmaxf(best, field_dot<PREC>(field, W, H, cx + dx, cy + dy, fx, fy));
                    aw[b * 3 + u] += best;
                    a1[b * 3 + u] += field_dot<PREC>(field, W, H, cx, cy, fx, fy);
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
            red[wv][m] = aw[m];
            red[wv][9 + m] = a1[m];
        }
    }
    __syncthreads();
    if (threadIdx.x < 18) {
        float s = 0.f;
        for (int w = 0; w < kWaves; ++w) s += red[w][threadIdx.x];
        P.part[l][(((size_t)c * 3 + g) * chunks + chunk) * 18 + threadIdx.x] = s;
    }
}

struct PickArgs {
    int K0, full, max_cand, src;
    double theta_min, step0;
};

// Pick of the level-0 poses after the last refinement launch, written over
// the candidates.  grid: (candidate, pair).
__global__ __launch_bounds__(64) void k_refine_pick(PickArgs a, const PairDesc* __restrict__ pairs)
{
    const PairDesc& P = pairs[blockIdx.y];
    const int c = blockIdx.x;
    int count = a.max_cand;
    if (P.ncand) count = min(count, *P.ncand);
    if (c >= count) return;
    const tm_pose ctr = P.ctr[a.src][c];
    float sw, s1;
    int x, y, k;
    pick27(P.part[0] + (size_t)c * 3 * chunks_of(P.n[0]) * 18, chunks_of(P.n[0]), ctr.x, ctr.y, ctr.k, P.W[0], P.H[0],
           P.n[0], a.K0, a.full, &sw, &s1, &x, &y, &k);
    if (threadIdx.x == 0) {
        tm_pose o;
        o.x = x;
        o.y = y;
        o.k = k;
        o.level = 0;
        o.theta_deg = (float)level_theta(a.theta_min, a.step0, k);
        o.score_w = sw;
        o.score_1 = s1;
        o.reserved = 0;
        P.cand[c] = o;
    }
}

}  // namespace

int refine_chunks(int n) { return (n + kThreads - 1) / kThreads; }

hipError_t launch_refine(const SearchDesc& s, const PairDesc* d, int npairs, int from_level, const int* max_chunks,
                         hipStream_t st)
{
    if (from_level <= 0 || npairs == 0) return hipSuccess;
    from_level = min(from_level, s.L - 1);
    int src = 0;
    for (int l = from_level - 1; l >= 0; --l) {
        LevelArgs a;
        a.level = l;
        a.max_chunks = max_chunks[l];
        a.pick = l < from_level - 1;
        a.K = s.K[l];
        a.K_above = s.K[l + 1];
        a.step = s.step[l];
        a.step_above = s.step[l + 1];
        a.full = s.full;
        a.win = s.win;
        a.max_cand = s.max_cand;
        a.theta_min = s.theta_min;
        a.src = src;
        dim3 grid((unsigned)(s.max_cand * 3 * a.max_chunks), npairs);
        if (s.precision == TM_FP16)
            hipLaunchKernelGGL(k_refine_level<TM_FP16>, grid, dim3(kThreads), 0, st, a, d);
        else
            hipLaunchKernelGGL(k_refine_level<TM_FP32>, grid, dim3(kThreads), 0, st, a, d);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        src ^= 1;
    }
    PickArgs pa;
    pa.K0 = s.K[0];
    pa.full = s.full;
    pa.max_cand = s.max_cand;
    pa.src = src;
    pa.theta_min = s.theta_min;
    pa.step0 = s.step[0];
    hipLaunchKernelGGL(k_refine_pick, dim3(s.max_cand, npairs), dim3(64), 0, st, pa, d);
    return hipGetLastError();
}

}  // namespace tmk
