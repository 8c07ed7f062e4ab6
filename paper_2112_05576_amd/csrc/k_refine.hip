// Coarse-to-fine refinement.  The paper starts the score computation at the
// top image of the pyramid (Sec. II para. 2); each candidate found there is
// carried down one level at a time by re-scoring the 27 poses
// (2x + a, 2y + b, 2k + c), a, b, c in {-1, 0, 1}, with the same windowed
// score (Eq. 1) and keeping the best by the selection key.
//
// One launch per level.  The grid is candidate x angle c x chunk of model
// points, so that a level spreads over hundreds of workgroups.  A workgroup
// first picks its candidate's pose at the level above from that level's
// partial sums (every workgroup of the candidate makes the same pick, in the
// same order), then forms q_i and r_i of its points in FP64, reads the 5x5
// field block covering the 3x3 windows of the 9 translations with all 25
// loads in flight, and accumulates 9 windowed votes and 9 centre votes.
// Sums are combined by a fixed butterfly per wave and in wave order across
// the workgroup, then across chunks in chunk order at the pick.
#include "tm_device.h"

namespace tmk {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Best of the 27 poses around `c` (a pose of level l+1) at level l, from the
// partial sums part[g][chunk][m] (m < 9: S_w of translation m, m >= 9: S_1).
// Runs on one wave; every lane returns the result.
__device__ void pick27(const float* __restrict__ part, int chunks, int x, int y, int k, const RefineLevel& L,
                       int full, float* bw, float* b1, int* bx, int* by, int* bk)
{
    const int lane = threadIdx.x & 63;
    const int m = lane < 27 ? lane : 26;
    const int g = m / 9, t = m % 9, b = t / 3, u = t % 3;
    const int kg = angle_index(2 * k + g - 1, L.K, full);
    const int xx = 2 * x + u - 1, yy = 2 * y + b - 1;
    float sw = 0.f, s1 = 0.f;
    for (int ch = 0; ch < chunks; ++ch) {
        const float* p = part + ((size_t)g * chunks + ch) * 18;
        sw += p[t];
        s1 += p[9 + t];
    }
    sw /= (float)L.n;
    s1 /= (float)L.n;
    const bool ok = lane < 27 && xx >= 0 && yy >= 0 && xx < L.W && yy < L.H;
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

struct LevelArgs {
    RefineLevel cur;       // level l being scored
    RefineLevel above;     // level l+1 (for the pick of its pose)
    int level;             // l
    int chunks;            // point chunks of level l
    int chunks_above;      // point chunks of level l+1 (0: no pick, poses are given)
    int full, win;
    double theta_min;
    const tm_pose* poses;  // given poses (when chunks_above == 0)
    const int32_t* n_dev;  // candidate count (device) or null
    int n;                 // candidate capacity
    tm_pose* centre_in;    // poses of level l+2 (centres of the pick), when chunks_above > 0
    tm_pose* centre_out;   // poses of level l+1 written here
    const float* part_above;  // [n][3][chunks_above][18]
    float* part;              // [n][3][chunks][18]
};

template <int PREC>
__global__ __launch_bounds__(kThreads) void k_refine_level(LevelArgs a)
{
    __shared__ float red[kWaves][18];
    __shared__ int cur[3];
    const int chunk = blockIdx.x % a.chunks;
    const int g = (blockIdx.x / a.chunks) % 3;
    const int c = blockIdx.x / (a.chunks * 3);
    int count = a.n;
    if (a.n_dev) count = min(count, *a.n_dev);
    if (c >= count) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    if (threadIdx.x < 64) {
        int x, y, k;
        float sw, s1;
        if (a.chunks_above > 0) {
            const tm_pose ctr = a.centre_in[c];
            pick27(a.part_above + (size_t)c * 3 * a.chunks_above * 18, a.chunks_above, ctr.x, ctr.y, ctr.k, a.above,
                   a.full, &sw, &s1, &x, &y, &k);
        } else {
            const tm_pose p = a.poses[c];
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
            if (blockIdx.x % (a.chunks * 3) == 0) {
                tm_pose o;
                o.x = x;
                o.y = y;
                o.k = k;
                o.level = a.level + 1;
                o.theta_deg = (float)level_theta(a.theta_min, a.above.step, k);
                o.score_w = sw;
                o.score_1 = s1;
                o.reserved = 0;
                a.centre_out[c] = o;
            }
        }
    }
    __syncthreads();
    const int x = cur[0], y = cur[1], k = cur[2];
    const RefineLevel& L = a.cur;
    const int kc = angle_index(2 * k + g - 1, L.K, a.full);
    double cs, sn;
    sincos_deg(level_theta(a.theta_min, L.step, kc), &cs, &sn);
    float aw[9], a1[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        aw[m] = 0.f;
        a1[m] = 0.f;
    }
    const int per = (L.n + a.chunks - 1) / a.chunks;
    const int i0 = chunk * per, i1 = min(L.n, i0 + per);
    const int wh = (a.win - 1) / 2;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += kThreads) {
        int qx, qy;
        double rx, ry;
        project_point(L.pts[i], cs, sn, &qx, &qy, &rx, &ry);
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
                cin[u] = (unsigned)xx < (unsigned)L.W;
                rin[u] = (unsigned)yy < (unsigned)L.H;
                col[u] = min(max(xx, 0), L.W - 1);
                rowoff[u] = (size_t)min(max(yy, 0), L.H - 1) * L.W;
            }
            float2 gv[5][5];
#pragma unroll
            for (int v = 0; v < 5; ++v)
#pragma unroll
                for (int u = 0; u < 5; ++u) gv[v][u] = field_load<PREC>(L.field, rowoff[v] + col[u]);
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
                            best = fmaxf(best, field_dot<PREC>(L.field, L.W, L.H, cx + dx, cy + dy, fx, fy));
                    aw[b * 3 + u] += best;
                    a1[b * 3 + u] += field_dot<PREC>(L.field, L.W, L.H, cx, cy, fx, fy);
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
        a.part[(((size_t)c * 3 + g) * a.chunks + chunk) * 18 + threadIdx.x] = s;
    }
}

// Pick of the level-0 poses after the last refinement launch.
__global__ __launch_bounds__(64) void k_refine_pick(RefineLevel L0, int full, double theta_min, const tm_pose* centre,
                                                     const float* __restrict__ part, int chunks,
                                                     const int32_t* n_dev, int n, tm_pose* out)
{
    const int c = blockIdx.x;
    int count = n;
    if (n_dev) count = min(count, *n_dev);
    if (c >= count) return;
    const tm_pose ctr = centre[c];
    float sw, s1;
    int x, y, k;
    pick27(part + (size_t)c * 3 * chunks * 18, chunks, ctr.x, ctr.y, ctr.k, L0, full, &sw, &s1, &x, &y, &k);
    if (threadIdx.x == 0) {
        tm_pose o;
        o.x = x;
        o.y = y;
        o.k = k;
        o.level = 0;
        o.theta_deg = (float)level_theta(theta_min, L0.step, k);
        o.score_w = sw;
        o.score_1 = s1;
        o.reserved = 0;
        out[c] = o;
    }
}

int chunks_for(int n) { return (n + kThreads - 1) / kThreads; }

}  // namespace

size_t refine_workspace_bytes(const RefineArgs& a, int n)
{
    size_t b = 2 * (size_t)n * sizeof(tm_pose);
    for (int l = 0; l < a.L; ++l) b += (size_t)n * 3 * chunks_for(a.lv[l].n) * 18 * sizeof(float);
    return b + 256;
}

hipError_t launch_refine(const RefineArgs& a, tm_pose* poses, int n, const int32_t* n_dev, int from_level, void* ws,
                         hipStream_t s)
{
    if (n == 0 || from_level <= 0) return hipSuccess;
    from_level = min(from_level, a.L - 1);
    uint8_t* base = reinterpret_cast<uint8_t*>(ws);
    tm_pose* ctr[2] = {reinterpret_cast<tm_pose*>(base), reinterpret_cast<tm_pose*>(base) + n};
    float* part[kMaxLevels];
    size_t off = 2 * (size_t)n * sizeof(tm_pose);
    for (int l = 0; l < a.L; ++l) {
        part[l] = reinterpret_cast<float*>(base + off);
        off += (size_t)n * 3 * chunks_for(a.lv[l].n) * 18 * sizeof(float);
    }
    int flip = 0;
    for (int l = from_level - 1; l >= 0; --l) {
        LevelArgs la;
        la.cur = a.lv[l];
        la.above = a.lv[l + 1];
        la.level = l;
        la.chunks = chunks_for(a.lv[l].n);
        la.chunks_above = (l == from_level - 1) ? 0 : chunks_for(a.lv[l + 1].n);
        la.full = a.full;
        la.win = a.win;
        la.theta_min = a.theta_min;
        la.poses = poses;
        la.n_dev = n_dev;
        la.n = n;
        la.centre_in = ctr[flip];
        la.centre_out = ctr[flip ^ 1];
        la.part_above = part[l + 1];
        la.part = part[l];
        dim3 grid((unsigned)(n * 3 * la.chunks));
        if (a.precision == TM_FP16)
            hipLaunchKernelGGL(k_refine_level<TM_FP16>, grid, dim3(kThreads), 0, s, la);
        else
            hipLaunchKernelGGL(k_refine_level<TM_FP32>, grid, dim3(kThreads), 0, s, la);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        flip ^= 1;
    }
    hipLaunchKernelGGL(k_refine_pick, dim3(n), dim3(64), 0, s, a.lv[0], a.full, a.theta_min, ctr[flip], part[0],
                       chunks_for(a.lv[0].n), n_dev, n, poses);
    return hipGetLastError();
}

}  // namespace tmk
