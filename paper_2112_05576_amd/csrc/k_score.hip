// Similarity score of Eq. (1) with the per-point neighbouring search
// (Sec. II paras. 3-5): the exhaustive pose search of one level and the
// scoring of arbitrary poses.
//
// Dense search layout.  A workgroup stages a tile of the direction field
// (plus a halo of the model's rotated radius + 1) in LDS, then each wave
// scores one angle at a time for a block of translations: lane j of a G-lane
// segment owns column X0 - 1 + j and an R-row strip.  For one model point the
// lane computes the dot product r_i . g of its own column on R + 2 rows, takes
// the vertical max of three rows, and gets the left and right columns' values
// from its neighbour lanes through wave-shift DPP, so a 3x3 window costs R + 2
// dot products instead of 9 R.  The two edge lanes of a segment only supply
// neighbour values; their own outputs are discarded.  Sums over points run in
// point order per lane, in blocks of 32 (bounding FP32 error by about
// 2^-24 (32 + n/32) per score).  Each workgroup covers a chunk of angles and
// writes its best angle per translation; a second kernel reduces the chunks.
#include <stdlib.h>

#include "tm_device.h"

namespace tmk {

namespace {

constexpr int kBlock = 32;  // points per partial sum

// Wave-wide shifts by one lane (DPP wave_shr:1 / wave_shl:1).  Lanes without
// a source read 0; they are the discarded edge lanes.
__device__ __forceinline__ float dpp_from_lower(float v)  // lane j receives lane j-1
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));
}

__device__ __forceinline__ float dpp_from_upper(float v)  // lane j receives lane j+1
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xF, 0xF, true));
}

struct FastArgs {
    const float2* field;
    int W, H;
    const TabEntry* tab;
    int n_pad, K;
    float n_f;
    int A;              // angles per workgroup
    int WY, WA;         // waves stacked in y, waves splitting the angles
    int tiles_x, tiles_y;
    int halo, LR;       // halo width, LDS rows
    float* pw;          // [C][H][W] partial best S_w
    float* p1;          //            partial best S_1
    int32_t* pk;        //            partial best k
};

template <int G, int R, int LC>
__global__ __launch_bounds__(1024) void k_dense_fast(FastArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float2* tile = reinterpret_cast<float2*>(smem);
    constexpr int NS = 64 / G;   // segments per wave
    constexpr int TW = G - 2;    // output columns per segment
    const int TH = a.WY * NS * R;
    const int n_tiles = a.tiles_x * a.tiles_y;
    const int chunk = blockIdx.x / n_tiles;
    const int tid = blockIdx.x % n_tiles;
    const int X0 = (tid % a.tiles_x) * TW, Y0 = (tid / a.tiles_x) * TH;
    const int halo = a.halo;
    const int fc = TW + 2 * halo;

    for (int e = threadIdx.x; e < a.LR * fc; e += blockDim.x) {
        const int r = e / fc, c = e - r * fc;
        const int x = X0 - halo + c, y = Y0 - halo + r;
        float2 v = make_float2(0.f, 0.f);
        if (x >= 0 && x < a.W && y >= 0 && y < a.H) v = a.field[(size_t)y * a.W + x];
        tile[r * LC + c] = v;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int wy = wid % a.WY, wa = wid / a.WY;
    const int seg = lane / G, li = lane - seg * G;
    const int row0 = (wy * NS + seg) * R;  // first output row of the strip, tile-relative
    const float2* lbase = tile + (halo - 1 + row0) * LC + (halo - 1 + li);

    float bw[R], b1[R];
    int bk[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        bw[r] = -INFINITY;
        b1[r] = -INFINITY;
        bk[r] = -1;
    }
    const int k0 = chunk * a.A, k1 = min(a.K, k0 + a.A);
    for (int k = k0 + wa; k < k1; k += a.WA) {
        const TabEntry* __restrict__ T = a.tab + (size_t)k * a.n_pad;
        float tw[R], t1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            tw[r] = 0.f;
            t1[r] = 0.f;
        }
        for (int i0 = 0; i0 < a.n_pad; i0 += kBlock) {
            float pw[R], p1[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                pw[r] = 0.f;
                p1[r] = 0.f;
            }
            const int i1 = min(a.n_pad, i0 + kBlock);
#pragma unroll 2
            for (int i = i0; i < i1; ++i) {
                const TabEntry e = T[i];
                const float2* p = lbase + (int)e.qy * LC + (int)e.qx;
                float D[R + 2];
#pragma unroll
                for (int rr = 0; rr < R + 2; ++rr) {
                    const float2 g = p[rr * LC];
                    D[rr] = e.rx * g.x + e.ry * g.y;
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float v = fmaxf(fmaxf(D[r], D[r + 1]), D[r + 2]);
                    pw[r] += fmaxf(fmaxf(v, dpp_from_lower(v)), dpp_from_upper(v));
                    p1[r] += D[r + 1];
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                tw[r] += pw[r];
                t1[r] += p1[r];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float sw = tw[r] / a.n_f, s1 = t1[r] / a.n_f;
            if (sw > bw[r] || (sw == bw[r] && s1 > b1[r])) {
                bw[r] = sw;
                b1[r] = s1;
                bk[r] = k;
            }
        }
    }

    // combine the WA waves that share this tile, in key order
    __syncthreads();
    const int npos = TH * TW;
    float* cw = reinterpret_cast<float*>(smem);
    float* c1 = cw + a.WA * npos;
    int* ck = reinterpret_cast<int*>(c1 + a.WA * npos);
    if (li >= 1 && li <= G - 2) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int idx = (wa * TH + row0 + r) * TW + (li - 1);
            cw[idx] = bw[r];
            c1[idx] = b1[r];
            ck[idx] = bk[r];
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < npos; p += blockDim.x) {
        const int py = p / TW, px = p - py * TW;
        const int X = X0 + px, Y = Y0 + py;
        if (X >= a.W || Y >= a.H) continue;
        float w0 = cw[p], s0 = c1[p];
        int kk = ck[p];
        for (int w = 1; w < a.WA; ++w) {
            const int q = w * npos + p;
            if (key_better(cw[q], c1[q], 0, 0, ck[q], w0, s0, 0, 0, kk)) {
                w0 = cw[q];
                s0 = c1[q];
                kk = ck[q];
            }
        }
        const size_t o = ((size_t)chunk * a.H + Y) * a.W + X;
        a.pw[o] = w0;
        a.p1[o] = s0;
        a.pk[o] = kk;
    }
}

struct GenericArgs {
    const void* field;
    int W, H, precision;
    const TabEntry* tab;
    int n, n_pad, K;
    float n_f;
    int sx, sy, win, gw, gh;
    int A;
    float* pw;
    float* p1;
    int32_t* pk;
};

// Any step and window: one thread per grid translation, taps read from
// global memory (clamped addresses, no branches).
template <int PREC>
__global__ __launch_bounds__(256) void k_dense_generic(GenericArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = blockIdx.y;
    if (p >= a.gw * a.gh) return;
    const int gy = p / a.gw, gx = p - gy * a.gw;
    const int x = gx * a.sx, y = gy * a.sy;
    const int h = (a.win - 1) / 2;
    float bw = -INFINITY, b1 = -INFINITY;
    int bk = -1;
    const int k0 = chunk * a.A, k1 = min(a.K, k0 + a.A);
    for (int k = k0; k < k1; ++k) {
        const TabEntry* __restrict__ T = a.tab + (size_t)k * a.n_pad;
        float tw = 0.f, t1 = 0.f;
        for (int i0 = 0; i0 < a.n; i0 += kBlock) {
            float pw = 0.f, p1 = 0.f;
            const int i1 = min(a.n, i0 + kBlock);
            for (int i = i0; i < i1; ++i) {
                const TabEntry e = T[i];
                const int px = x + e.qx, py = y + e.qy;
                float best = -INFINITY;
                for (int dy = -h; dy <= h; ++dy)
#pragma unroll 3
                    for (int dx = -h; dx <= h; ++dx)
                        best = fmaxf(best, field_dot<PREC>(a.field, a.W, a.H, px + dx, py + dy, e.rx, e.ry));
                pw += best;
                p1 += field_dot<PREC>(a.field, a.W, a.H, px, py, e.rx, e.ry);
            }
            tw += pw;
            t1 += p1;
        }
        const float sw = tw / a.n_f, s1 = t1 / a.n_f;
        if (sw > bw || (sw == bw && s1 > b1)) {
            bw = sw;
            b1 = s1;
            bk = k;
        }
    }
    const size_t o = ((size_t)chunk * a.gh + gy) * a.gw + gx;
    a.pw[o] = bw;
    a.p1[o] = b1;
    a.pk[o] = bk;
}

// Best angle per translation over the C chunk partials, in key order.  A
// workgroup takes 32 translations; 8 threads share one translation, each
// scanning every 8th chunk with its loads issued ahead of the comparisons,
// then the 8 partial bests are merged through LDS.  The key is a total order,
// so the result does not depend on the split.
constexpr int kRedLanes = 8;
constexpr int kRedPos = 32;

__global__ __launch_bounds__(256) void k_reduce_chunks(const float* __restrict__ pw, const float* __restrict__ p1,
                                                        const int32_t* __restrict__ pk, int C, int np,
                                                        float* __restrict__ ow, float* __restrict__ o1,
                                                        int32_t* __restrict__ ok)
{
    __shared__ float sw_[kRedPos][kRedLanes], s1_[kRedPos][kRedLanes];
    __shared__ int sk_[kRedPos][kRedLanes];
    const int lane = threadIdx.x % kRedLanes, slot = threadIdx.x / kRedLanes;
    const int p = blockIdx.x * kRedPos + slot;
    float w0 = -INFINITY, s0 = -INFINITY;
    int k = 0x7fffffff;
    if (p < np) {
        int c = lane;
        for (; c + 3 * kRedLanes < C; c += 4 * kRedLanes) {
            float w[4], s[4];
            int kk[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const size_t q = (size_t)(c + u * kRedLanes) * np + p;
                w[u] = pw[q];
                s[u] = p1[q];
                kk[u] = pk[q];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (key_better(w[u], s[u], 0, 0, kk[u], w0, s0, 0, 0, k)) {
                    w0 = w[u];
                    s0 = s[u];
                    k = kk[u];
                }
        }
        for (; c < C; c += kRedLanes) {
            const size_t q = (size_t)c * np + p;
            const float w = pw[q], s = p1[q];
            const int kk = pk[q];
            if (key_better(w, s, 0, 0, kk, w0, s0, 0, 0, k)) {
                w0 = w;
                s0 = s;
                k = kk;
            }
        }
    }
    sw_[slot][lane] = w0;
    s1_[slot][lane] = s0;
    sk_[slot][lane] = k;
    __syncthreads();
    if (lane == 0 && p < np) {
        for (int u = 1; u < kRedLanes; ++u)
            if (key_better(sw_[slot][u], s1_[slot][u], 0, 0, sk_[slot][u], w0, s0, 0, 0, k)) {
                w0 = sw_[slot][u];
                s0 = s1_[slot][u];
                k = sk_[slot][u];
            }
        ow[p] = w0;
        o1[p] = s0;
        ok[p] = k;
    }
}

// One wave per pose: lanes take points i = lane, lane + 64, ...; each point's
// rotation is formed in FP64, its window read from global memory; per-lane
// sums are combined by a fixed butterfly.
template <int PREC>
__global__ __launch_bounds__(256) void k_sparse(const void* __restrict__ field, int W, int H,
                                                 const ModelPoint* __restrict__ pts, int n, int win,
                                                 const tm_eval_pose* __restrict__ poses, int np,
                                                 float* __restrict__ scores)
{
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= np) return;
    const tm_eval_pose ps = poses[w];
    double c, s;
    sincos_deg(ps.theta_deg, &c, &s);
    const int h = (win - 1) / 2;
    float sw = 0.f, s1 = 0.f;
    for (int i = lane; i < n; i += 64) {
        int qx, qy;
        double rx, ry;
        project_point(pts[i], c, s, &qx, &qy, &rx, &ry);
        const float fx = (float)rx, fy = (float)ry;
        const int px = ps.x + qx, py = ps.y + qy;
        float best = -INFINITY;
        for (int dy = -h; dy <= h; ++dy)
#pragma unroll 3
            for (int dx = -h; dx <= h; ++dx)
                best = fmaxf(best, field_dot<PREC>(field, W, H, px + dx, py + dy, fx, fy));
        sw += best;
        s1 += field_dot<PREC>(field, W, H, px, py, fx, fy);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sw += __shfl_xor(sw, off, 64);
        s1 += __shfl_xor(s1, off, 64);
    }
    if (lane == 0) {
        scores[2 * w] = sw / (float)n;
        scores[2 * w + 1] = s1 / (float)n;
    }
}

// ---------------------------------------------------------------- planning
struct Plan {
    bool fast;
    int G, R, LC;
    int WY, WA;
    int tiles_x, tiles_y;
    int halo, LR;
    int A, C;
    size_t lds;
};

constexpr int kLC[] = {64, 96, 128, 192, 256};

// Launch-shape knobs of the search kernel: waves stacked in y per workgroup,
// waves splitting the angle chunk, and angles per wave.  Defaults can be
// overridden by TM_DENSE_WY / TM_DENSE_WA / TM_DENSE_APW (tuning runs).
int knob(const char* name, int dflt, int lo, int hi)
{
    const char* v = getenv(name);
    if (!v || !*v) return dflt;
    int x = atoi(v);
    return x < lo ? lo : (x > hi ? hi : x);
}

Plan make_plan(const DenseGeom& g)
{
    Plan p = {};
    const int halo = g.rad + 1;
    p.fast = g.sx == 1 && g.sy == 1 && g.win == 3 && g.precision == TM_FP32;
    if (p.fast) {
        p.G = 32;
        p.R = 8;
        p.WY = knob("TM_DENSE_WY", 1, 1, 4);
        p.WA = knob("TM_DENSE_WA", 4, 1, 16);
        if (p.WY * p.WA > 16) p.WA = 16 / p.WY;
        const int TW = p.G - 2, TH = p.WY * (64 / p.G) * p.R;
        p.LC = 0;
        for (int lc : kLC)
            if (lc >= TW + 2 * halo) {
                p.LC = lc;
                break;
            }
        p.halo = halo;
        p.LR = TH + 2 * halo;
        p.tiles_x = (g.W + TW - 1) / TW;
        p.tiles_y = (g.H + TH - 1) / TH;
        size_t tile_bytes = (size_t)p.LR * p.LC * sizeof(float2);
        size_t comb_bytes = (size_t)12 * p.WA * TH * TW;
        p.lds = tile_bytes > comb_bytes ? tile_bytes : comb_bytes;
        if (p.LC == 0 || p.lds > 160 * 1024) p.fast = false;
    }
    if (p.fast) {
        // about four waves per SIMD over the whole grid, whole angles per wave
        const long long units = (long long)p.tiles_x * p.tiles_y * g.K;
        long long per_wave = units / 4096;
        if (per_wave < 1) per_wave = 1;
        per_wave = knob("TM_DENSE_APW", (int)per_wave, 1, 1 << 20);
        p.A = (int)(per_wave * p.WA);
        p.C = (g.K + p.A - 1) / p.A;
    } else {
        const int blocks = (g.gw * g.gh + 255) / 256;
        int C = (2048 + blocks - 1) / blocks;  // enough workgroups to fill the chip
        if (C > g.K) C = g.K;
        if (C < 1) C = 1;
        p.A = (g.K + C - 1) / C;
        p.C = (g.K + p.A - 1) / p.A;
    }
    return p;
}

template <int G, int R, int LC>
hipError_t launch_fast_t(const Plan& p, const FastArgs& a, hipStream_t s)
{
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_fast<G, R, LC>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int blocks = p.tiles_x * p.tiles_y * p.C;
    hipLaunchKernelGGL((k_dense_fast<G, R, LC>), dim3(blocks), dim3(64 * p.WY * p.WA), p.lds, s, a);
    return hipGetLastError();
}

hipError_t launch_fast(const Plan& p, const FastArgs& a, hipStream_t s)
{
    switch (p.LC) {
        case 64: return launch_fast_t<32, 8, 64>(p, a, s);
        case 96: return launch_fast_t<32, 8, 96>(p, a, s);
        case 128: return launch_fast_t<32, 8, 128>(p, a, s);
        case 192: return launch_fast_t<32, 8, 192>(p, a, s);
        default: return launch_fast_t<32, 8, 256>(p, a, s);
    }
}

}  // namespace

size_t dense_workspace_bytes(const DenseGeom& g)
{
    Plan p = make_plan(g);
    const size_t np = p.fast ? (size_t)g.W * g.H : (size_t)g.gw * g.gh;
    return (size_t)p.C * np * 12 + 256;
}

hipError_t launch_dense(const DenseGeom& g, void* ws, float* ow, float* o1, int32_t* ok, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1)
{
    Plan p = make_plan(g);
    const size_t np = p.fast ? (size_t)g.W * g.H : (size_t)g.gw * g.gh;
    float* pw = reinterpret_cast<float*>(ws);
    float* p1 = pw + (size_t)p.C * np;
    int32_t* pk = reinterpret_cast<int32_t*>(p1 + (size_t)p.C * np);
    hipError_t e;
    if (ev0) {
        e = hipEventRecord(ev0, s);
        if (e != hipSuccess) return e;
    }
    if (p.fast) {
        FastArgs a;
        a.field = reinterpret_cast<const float2*>(g.field);
        a.W = g.W;
        a.H = g.H;
        a.tab = g.tab;
        a.n_pad = g.n_pad;
        a.K = g.K;
        a.n_f = (float)g.n;
        a.A = p.A;
        a.WY = p.WY;
        a.WA = p.WA;
        a.tiles_x = p.tiles_x;
        a.tiles_y = p.tiles_y;
        a.halo = p.halo;
        a.LR = p.LR;
        a.pw = pw;
        a.p1 = p1;
        a.pk = pk;
        e = launch_fast(p, a, s);
    } else {
        GenericArgs a;
        a.field = g.field;
        a.W = g.W;
        a.H = g.H;
        a.precision = g.precision;
        a.tab = g.tab;
        a.n = g.n;
        a.n_pad = g.n_pad;
        a.K = g.K;
        a.n_f = (float)g.n;
        a.sx = g.sx;
        a.sy = g.sy;
        a.win = g.win;
        a.gw = g.gw;
        a.gh = g.gh;
        a.A = p.A;
        a.pw = pw;
        a.p1 = p1;
        a.pk = pk;
        dim3 grid((g.gw * g.gh + 255) / 256, p.C);
        if (g.precision == TM_FP16)
            hipLaunchKernelGGL(k_dense_generic<TM_FP16>, grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL(k_dense_generic<TM_FP32>, grid, dim3(256), 0, s, a);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (ev1) {
        e = hipEventRecord(ev1, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)((np + kRedPos - 1) / kRedPos)), dim3(kRedPos * kRedLanes), 0,
                       s, pw, p1, pk, p.C,
                       (int)np, ow, o1, ok);
    return hipGetLastError();
}

hipError_t launch_sparse(const void* field, int W, int H, int precision, const ModelPoint* pts, int n, int win,
                         const tm_eval_pose* poses, int np, float* scores, hipStream_t s)
{
    if (np == 0) return hipSuccess;
    if (precision == TM_FP16)
        hipLaunchKernelGGL(k_sparse<TM_FP16>, dim3((np + 3) / 4), dim3(256), 0, s, field, W, H, pts, n, win, poses,
                           np, scores);
    else
        hipLaunchKernelGGL(k_sparse<TM_FP32>, dim3((np + 3) / 4), dim3(256), 0, s, field, W, H, pts, n, win, poses,
                           np, scores);
    return hipGetLastError();
}

}  // namespace tmk
