// Device-side helpers shared by the kernels: degree sine/cosine, the rigid
// projection of one model point (Eq. 2), field loads and the selection key.
#pragma once

#include "tm_internal.h"

namespace tmk {

// cos and sin of an angle in degrees with an exact reduction to the first
// quadrant, so that every multiple of 90 degrees yields exact 0 and +-1 and a
// quarter turn of the angle is an exact swap/negation of the pair.
__device__ __forceinline__ void sincos_deg(double deg, double* c, double* s)
{
#pragma clang fp contract(off)
    double r = fmod(deg, 360.0);
    if (r < 0.0) r += 360.0;
    if (r >= 360.0) r -= 360.0;
    int q = (int)floor(r / 90.0);
    q = q > 3 ? 3 : q;
    double phi = r - 90.0 * (double)q;
    double rad = phi * (M_PI / 180.0);
    double c0 = cos(rad), s0 = sin(rad);
    if (q == 0) { *c = c0;  *s = s0; }
    else if (q == 1) { *c = -s0; *s = c0; }
    else if (q == 2) { *c = -c0; *s = -s0; }
    else { *c = s0; *s = -c0; }
}

// Eq. (2) for one model point without the translation: integer position
// offset q = floor(R t + 0.5 + 1e-9) (FP64, products rounded separately) and
// rotated unit direction r = R d, d = g / |g| formed in FP64.
__device__ __forceinline__ void project_point(const ModelPoint& p, double c, double s, int* qx, int* qy,
                                              double* rx, double* ry)
{
#pragma clang fp contract(off)
    double tx = (double)p.tx, ty = (double)p.ty;
    double vx = c * tx - s * ty;
    double vy = s * tx + c * ty;
    *qx = (int)floor(vx + 0.5 + 1e-9);
    *qy = (int)floor(vy + 0.5 + 1e-9);
    double gx = (double)p.gx, gy = (double)p.gy;
    double m = sqrt(gx * gx + gy * gy);
    double dx = gx / m, dy = gy / m;
    *rx = c * dx - s * dy;
    *ry = s * dx + c * dy;
}

// The model point's unit direction d = g / |g| in FP64 (the same operations
// as in project_point, so a stored copy gives the same bits).
__device__ __forceinline__ void unit_dir(const ModelPoint& p, double* dx, double* dy)
{
#pragma clang fp contract(off)
    double gx = (double)p.gx, gy = (double)p.gy;
    double m = sqrt(gx * gx + gy * gy);
    *dx = gx / m;
    *dy = gy / m;
}

// The similarity projection with the unit direction given: q = floor(sigma
// (R t) + 0.5 + 1e-9), the rotation first and then the product with sigma
// (rounded separately), and r = R d.
__device__ __forceinline__ void project_dir_s(const ModelPoint& p, double dx, double dy, double c, double s,
                                              double sigma, int* qx, int* qy, double* rx, double* ry)
{
#pragma clang fp contract(off)
    double tx = (double)p.tx, ty = (double)p.ty;
    double vx = c * tx - s * ty;
    double vy = s * tx + c * ty;
    vx = sigma * vx;
    vy = sigma * vy;
    *qx = (int)floor(vx + 0.5 + 1e-9);
    *qy = (int)floor(vy + 0.5 + 1e-9);
    *rx = c * dx - s * dy;
    *ry = s * dx + c * dy;
}

// The similarity projection of a model point.  sigma == 1 gives
// project_point exactly.
__device__ __forceinline__ void project_point_s(const ModelPoint& p, double c, double s, double sigma, int* qx,
                                                int* qy, double* rx, double* ry)
{
    double dx, dy;
    unit_dir(p, &dx, &dy);
    project_dir_s(p, dx, dy, c, s, sigma, qx, qy, rx, ry);
}

// Scale j of the grid sigma_min + j * sigma_step.
__device__ __forceinline__ double scale_of(double sigma_min, double sigma_step, int j)
{
#pragma clang fp contract(off)
    return sigma_min + (double)j * sigma_step;
}

__device__ __forceinline__ double level_theta(double theta_min, double step, int k)
{
#pragma clang fp contract(off)
    return theta_min + (double)k * step;
}

// Angle index on a level grid: wrap for a full circle, clamp otherwise.
__device__ __forceinline__ int angle_index(int k, int K, int full)
{
    if (full) {
        int m = k % K;
        return m < 0 ? m + K : m;
    }
    return k < 0 ? 0 : (k > K - 1 ? K - 1 : k);
}

// Direction field element as float2, for FP32 or FP16 storage.
template <int PREC>
__device__ __forceinline__ float2 field_load(const void* field, size_t o)
{
    if constexpr (PREC == TM_FP16) {
        return __half22float2(reinterpret_cast<const __half2*>(field)[o]);
    } else {
        return reinterpret_cast<const float2*>(field)[o];
    }
}

// Dot of a rotated model direction with the field at (x, y); 0 outside the
// image (and at non-edge pixels, whose stored direction is (0, 0)).  The
// address is clamped and the result selected, without a branch, so that the
// loads of many taps are in flight together.
template <int PREC>
__device__ __forceinline__ float field_dot(const void* field, int W, int H, int x, int y, float rx, float ry)
{
    const bool in = (unsigned)x < (unsigned)W && (unsigned)y < (unsigned)H;
    const int xc = min(max(x, 0), W - 1), yc = min(max(y, 0), H - 1);
    const float2 g = field_load<PREC>(field, (size_t)yc * W + xc);
    const float v = rx * g.x + ry * g.y;
    return in ? v : 0.0f;
}

// Edge-taps-only window (tm_vote TM_VOTE_EDGE).  A tap off the edge set
// (stored direction (0, 0)) or outside the image enters the window maximum as
// kOffEdge = -2, below every cosine; a maximum of -2 (no edge tap) then votes
// 0.  vote_finish does that by clearing bit 30 of the FP32 pattern: -2.0f is
// 0xC0000000 and becomes -0.0f, while every cosine has |v| < 2 (unit vectors,
// FP16 rounding included), so its bit 30 is clear and it passes unchanged.
constexpr float kOffEdge = -2.0f;

__device__ __forceinline__ float vote_finish(float m) { return __int_as_float(__float_as_int(m) & (int)0xBFFFFFFF); }

__device__ __forceinline__ bool on_edge(float2 g) { return g.x != 0.0f || g.y != 0.0f; }

// A window operand of the edge-taps reading at (x, y): the cosine on the edge
// set, kOffEdge elsewhere.
template <int PREC>
__device__ __forceinline__ float field_vote_tap(const void* field, int W, int H, int x, int y, float rx, float ry)
{
    const bool in = (unsigned)x < (unsigned)W && (unsigned)y < (unsigned)H;
    const int xc = min(max(x, 0), W - 1), yc = min(max(y, 0), H - 1);
    const float2 g = field_load<PREC>(field, (size_t)yc * W + xc);
    const float v = rx * g.x + ry * g.y;
    return in && on_edge(g) ? v : kOffEdge;
}

// Window operand under either reading (VOTE 0: all taps, 1: edge taps).
template <int PREC, int VOTE>
__device__ __forceinline__ float field_win_tap(const void* field, int W, int H, int x, int y, float rx, float ry)
{
    if constexpr (VOTE == 1)
        return field_vote_tap<PREC>(field, W, H, x, y, rx, ry);
    else
        return field_dot<PREC>(field, W, H, x, y, rx, ry);
}

template <int VOTE>
__device__ __forceinline__ float win_finish(float m)
{
    if constexpr (VOTE == 1)
        return vote_finish(m);
    else
        return m;
}

// The selection key: S_w desc, S_1 desc, then position x asc, y asc, then
// angle index asc.  true iff (aw, a1, ax, ay, ak) ranks strictly before b.
__device__ __forceinline__ bool key_better(float aw, float a1, int ax, int ay, int ak, float bw, float b1, int bx,
                                           int by, int bk)
{
    if (aw != bw) return aw > bw;
    if (a1 != b1) return a1 > b1;
    if (ax != bx) return ax < bx;
    if (ay != by) return ay < by;
    return ak < bk;
}

// The workgroup's place in a grid renumbered so that each XCD takes one
// contiguous run of it: workgroups go to the 8 XCDs in turn by their linear
// index (x fastest, then y, then z), so without this neighbouring blocks sit
// in different L2s and fetch their shared rows once per XCD.  A bijection of
// the grid (XCD k runs the k-th run, of q or q + 1 blocks).
constexpr unsigned kXcds = 8;
__device__ __forceinline__ uint3 xcd_block()
{
    const unsigned nx = gridDim.x, ny = gridDim.y;
    const unsigned total = nx * ny * gridDim.z;
    const unsigned lin = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    const unsigned q = total / kXcds, r = total % kXcds;
    const unsigned x = lin % kXcds, local = lin / kXcds;
    const unsigned m = x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
    return make_uint3(m % nx, m / nx % ny, m / (nx * ny));
}

// Best of the 27 poses around (x, y, k) (a pose of level l+1) at level l, from
// the per-wave sums part[g][w][m] (m < 9: S_w of translation m, m >= 9: S_1),
// the waves added in order.  Runs on LANES (64 or 32) aligned lanes of one
// wave; every one of them returns the result.
template <int LANES = 64>
__device__ __forceinline__ void pick27(const float* __restrict__ part, int x, int y, int k, int W, int H, int n, int K, int full,
                       float* bw, float* b1, int* bx, int* by, int* bk)
{
    static_assert(LANES == 64 || LANES == 32, "a wave or half a wave");
    const int lane = threadIdx.x & (LANES - 1);
    const int m = lane < 27 ? lane : 26;
    const int g = m / 9, t = m % 9, b = t / 3, u = t % 3;
    const int kg = angle_index(2 * k + g - 1, K, full);
    const int xx = 2 * x + u - 1, yy = 2 * y + b - 1;
    float aw = 0.f, a1 = 0.f;
#pragma unroll
    for (int w = 0; w < kRefineWaves; ++w) {
        aw += part[(g * kRefineWaves + w) * 18 + t];
        a1 += part[(g * kRefineWaves + w) * 18 + 9 + t];
    }
    const float sw = aw / (float)n;
    const float s1 = a1 / (float)n;
    const bool ok = lane < 27 && xx >= 0 && yy >= 0 && xx < W && yy < H;
    float kw = ok ? sw : -INFINITY, k1 = ok ? s1 : -INFINITY;
    int kx = ok ? xx : 0x7fffffff, ky = ok ? yy : 0x7fffffff, kk = ok ? kg : 0x7fffffff;
#pragma unroll
    for (int off = LANES / 2; off >= 1; off >>= 1) {
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

}  // namespace tmk
