// Continuous score, beside the paper's Eq. (1): the mean over the model's
// points of r_i . B(R(theta) t_i + u), B the bilinear interpolation of the
// unit-direction field (zero off the edge set and outside), without the
// neighbourhood window and without rounding positions, so that it can be
// differentiated with respect to the pose (u_x, u_y, theta in degrees):
//   d/du     = J_B(p)^T r,
//   d/dtheta = (pi/180) [ (R' d) . B(p) + r . (J_B(p) R' t) ],
// with R' the derivative of R by the angle in radians and J_B the Jacobian
// of B in the pixel cell containing p.
//
// One wave per pose, lanes over the model's points, a fixed butterfly for the
// sums.  Forward and backward are separate kernels (the backward multiplies
// by the upstream gradient); a third form evaluates the score in FP64 at
// several step lengths along a direction, for the final line search.
#include "tm_device.h"

namespace tmk {

namespace {

constexpr int kMaxAlphas = 16;

struct ContArgs {
    int level;
    int n;            // poses
    int batched;      // pose.pair selects the descriptor (else descriptor 0)
    int npairs;       // descriptors; a pose naming another pair gets NaN results
    int n_alpha;      // line search: step lengths
    double alpha[kMaxAlphas];
};

template <typename A>
__device__ __forceinline__ A wave_sum(A v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// A pose moved by alpha * dir, rounded to the FP32 pose record, so that the
// line search scores exactly the pose it returns.
__device__ __forceinline__ tm_cont_pose moved(tm_cont_pose p, double alpha, const float* dir)
{
    p.x = (float)((double)p.x + alpha * (double)dir[0]);
    p.y = (float)((double)p.y + alpha * (double)dir[1]);
    p.theta_deg = (float)((double)p.theta_deg + alpha * (double)dir[2]);
    return p;
}

// MODE 0: forward (FP32), out[pose] = S.  MODE 1: backward (FP32),
// out[3 pose + j] = gin[pose] dS/dpose_j.  MODE 2: FP64 score at pose +
// alpha_j dir, out64[pose * n_alpha + j].
template <int PREC, int MODE>
__global__ __launch_bounds__(256) void k_cont(ContArgs a, const PairDesc* __restrict__ pairs,
                                               const tm_cont_pose* __restrict__ poses, const float* __restrict__ dirs,
                                               const float* __restrict__ gin, float* __restrict__ out,
                                               double* __restrict__ out64)
{
    using Acc = typename std::conditional<MODE == 2, double, float>::type;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int pi = MODE == 2 ? w / a.n_alpha : w;
    const int j = MODE == 2 ? w % a.n_alpha : 0;
    if (pi >= a.n) return;
    const tm_cont_pose ps = poses[pi];
    const int pr = a.batched ? ps.pair : 0;
    if ((unsigned)pr >= (unsigned)a.npairs) {
        if (lane == 0) {
            const float nan = __builtin_nanf("");
            if (MODE == 0) out[pi] = nan;
            if (MODE == 1) out[3 * pi] = out[3 * pi + 1] = out[3 * pi + 2] = nan;
            if (MODE == 2) out64[w] = __builtin_nan("");
        }
        return;
    }
    const PairDesc& P = pairs[pr];
    double x = ps.x, y = ps.y, th = ps.theta_deg;
    if (MODE == 2) {
        const tm_cont_pose m = moved(ps, a.alpha[j], dirs + 3 * pi);
        x = m.x;
        y = m.y;
        th = m.theta_deg;
    }
    double c, s;
    sincos_deg(th, &c, &s);
    const int l = a.level;
    const void* field = P.field[l];
    const int W = P.W[l], H = P.H[l], n = P.n[l];
    const ModelPoint* __restrict__ pts = P.pts[l];
    const double2* __restrict__ dir = P.dir[l];  // g / |g| in FP64, stored with the model
    Acc sv = 0, gx = 0, gy = 0, gt = 0;
    for (int i = lane; i < n; i += 64) {
        const ModelPoint q = pts[i];
        const double tx = q.tx, ty = q.ty;
        const double2 d = dir[i];
        const double dx = d.x, dy = d.y;
        const double px = c * tx - s * ty + x, py = s * tx + c * ty + y;
        const double x0 = floor(px), y0 = floor(py);
        const Acc fx = (Acc)(px - x0), fy = (Acc)(py - y0);
        const int ix = (int)x0, iy = (int)y0;
        float2 f[2][2];
        bool in[2][2];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int xx = ix + u, yy = iy + b;
                in[b][u] = (unsigned)xx < (unsigned)W && (unsigned)yy < (unsigned)H;
                f[b][u] = field_load<PREC>(field, (size_t)min(max(yy, 0), H - 1) * W + min(max(xx, 0), W - 1));
            }
        Acc gx00 = in[0][0] ? (Acc)f[0][0].x : 0, gy00 = in[0][0] ? (Acc)f[0][0].y : 0;
        Acc gx10 = in[0][1] ? (Acc)f[0][1].x : 0, gy10 = in[0][1] ? (Acc)f[0][1].y : 0;
        Acc gx01 = in[1][0] ? (Acc)f[1][0].x : 0, gy01 = in[1][0] ? (Acc)f[1][0].y : 0;
        Acc gx11 = in[1][1] ? (Acc)f[1][1].x : 0, gy11 = in[1][1] ? (Acc)f[1][1].y : 0;
        const Acc rx = (Acc)(c * dx - s * dy), ry = (Acc)(s * dx + c * dy);
        const Acc bx = (1 - fx) * (1 - fy) * gx00 + fx * (1 - fy) * gx10 + (1 - fx) * fy * gx01 + fx * fy * gx11;
        const Acc by = (1 - fx) * (1 - fy) * gy00 + fx * (1 - fy) * gy10 + (1 - fx) * fy * gy01 + fx * fy * gy11;
        if (MODE != 1) {
            sv += rx * bx + ry * by;
        } else {
            const Acc bxx = (1 - fy) * (gx10 - gx00) + fy * (gx11 - gx01);
            const Acc byx = (1 - fy) * (gy10 - gy00) + fy * (gy11 - gy01);
            const Acc bxy = (1 - fx) * (gx01 - gx00) + fx * (gx11 - gx10);
            const Acc byy = (1 - fx) * (gy01 - gy00) + fx * (gy11 - gy10);
            const Acc dpx = rx * bxx + ry * byx, dpy = rx * bxy + ry * byy;
            const Acc rtx = (Acc)(-s * tx - c * ty), rty = (Acc)(c * tx - s * ty);
            const Acc rdx = (Acc)(-s * dx - c * dy), rdy = (Acc)(c * dx - s * dy);
            gx += dpx;
            gy += dpy;
            gt += (rdx * bx + rdy * by) + (rtx * dpx + rty * dpy);
        }
    }
    const Acc nf = (Acc)n;
    if (MODE != 1) {
        sv = wave_sum(sv);
        if (lane == 0) {
            if (MODE == 0)
                out[pi] = (float)(sv / nf);
            else
                out64[w] = (double)sv / (double)n;
        }
    } else {
        gx = wave_sum(gx);
        gy = wave_sum(gy);
        gt = wave_sum(gt);
        if (lane == 0) {
            const float g0 = gin ? gin[pi] : 1.0f;
            out[3 * pi] = g0 * (float)(gx / nf);
            out[3 * pi + 1] = g0 * (float)(gy / nf);
            out[3 * pi + 2] = g0 * (float)((Acc)(M_PI / 180.0) * gt / nf);
        }
    }
}

// Best step length per pose (score desc, then the earlier step), pose moved.
__global__ __launch_bounds__(256) void k_line_pick(ContArgs a, const double* __restrict__ s64,
                                                    tm_cont_pose* __restrict__ poses, const float* __restrict__ dirs,
                                                    float* __restrict__ scores)
{
    const int pi = blockIdx.x * blockDim.x + threadIdx.x;
    if (pi >= a.n) return;
    const int pr = a.batched ? poses[pi].pair : 0;
    if ((unsigned)pr >= (unsigned)a.npairs) {  // pose left as it is
        if (scores) scores[pi] = __builtin_nanf("");
        return;
    }
    int best = 0;
    double bs = s64[(size_t)pi * a.n_alpha];
    for (int j = 1; j < a.n_alpha; ++j) {
        const double v = s64[(size_t)pi * a.n_alpha + j];
        if (v > bs) {
            bs = v;
            best = j;
        }
    }
    poses[pi] = moved(poses[pi], a.alpha[best], dirs + 3 * pi);
    if (scores) scores[pi] = (float)bs;
}

ContArgs cont_args(int level, int n, int batched, int npairs)
{
    ContArgs a = {};
    a.level = level;
    a.n = n;
    a.batched = batched;
    a.npairs = batched ? npairs : 1;
    a.n_alpha = 1;
    return a;
}

}  // namespace

hipError_t launch_cont(const PairDesc* d, int batched, int npairs, int level, int precision, const tm_cont_pose* poses,
                       int n, const float* gin, float* out, bool backward, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    ContArgs a = cont_args(level, n, batched, npairs);
    dim3 grid((n + 3) / 4);
    if (backward) {
        if (precision == TM_FP16)
            hipLaunchKernelGGL((k_cont<TM_FP16, 1>), grid, dim3(256), 0, s, a, d, poses, nullptr, gin, out, nullptr);
        else
            hipLaunchKernelGGL((k_cont<TM_FP32, 1>), grid, dim3(256), 0, s, a, d, poses, nullptr, gin, out, nullptr);
    } else {
        if (precision == TM_FP16)
            hipLaunchKernelGGL((k_cont<TM_FP16, 0>), grid, dim3(256), 0, s, a, d, poses, nullptr, nullptr, out,
                               nullptr);
        else
            hipLaunchKernelGGL((k_cont<TM_FP32, 0>), grid, dim3(256), 0, s, a, d, poses, nullptr, nullptr, out,
                               nullptr);
    }
    return hipGetLastError();
}

size_t line_search_scratch_bytes(int n, int n_alpha) { return (size_t)n * n_alpha * sizeof(double) + 256; }

hipError_t launch_line_search(const PairDesc* d, int batched, int npairs, int level, int precision,
                              tm_cont_pose* poses, const float* dirs, int n, const double* alphas, int n_alpha,
                              float* scores, double* scratch, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    ContArgs a = cont_args(level, n, batched, npairs);
    a.n_alpha = n_alpha;
    for (int j = 0; j < n_alpha; ++j) a.alpha[j] = alphas[j];
    dim3 grid((unsigned)(((long long)n * n_alpha + 3) / 4));
    if (precision == TM_FP16)
        hipLaunchKernelGGL((k_cont<TM_FP16, 2>), grid, dim3(256), 0, s, a, d, poses, dirs, nullptr, nullptr, scratch);
    else
        hipLaunchKernelGGL((k_cont<TM_FP32, 2>), grid, dim3(256), 0, s, a, d, poses, dirs, nullptr, nullptr, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_line_pick, dim3((n + 255) / 256), dim3(256), 0, s, a, scratch, poses, dirs, scores);
    return hipGetLastError();
}

}  // namespace tmk
