// Selection of poses from scores.  The paper keeps the single best pose of
// the search (Sec. II para. 3: a pose is recorded when its score is better);
// for several instances this becomes: strict local maxima of the key
// (S_w desc, S_1 desc, x asc, y asc, k asc) on the translation grid above a
// score floor, sorted by the key, then greedy suppression of poses closer
// than a minimum level-0 distance to an already accepted one.
#include "tm_device.h"

namespace tmk {

namespace {

struct Keys {
    float* sw;
    float* s1;
    int* x;
    int* y;
    int* k;
};

__device__ __forceinline__ bool kb(const Keys& a, int i, int j)
{
    return key_better(a.sw[i], a.s1[i], a.x[i], a.y[i], a.k[i], a.sw[j], a.s1[j], a.x[j], a.y[j], a.k[j]);
}

__device__ __forceinline__ void kswap(const Keys& a, int i, int j)
{
    float t;
    int u;
    t = a.sw[i]; a.sw[i] = a.sw[j]; a.sw[j] = t;
    t = a.s1[i]; a.s1[i] = a.s1[j]; a.s1[j] = t;
    u = a.x[i]; a.x[i] = a.x[j]; a.x[j] = u;
    u = a.y[i]; a.y[i] = a.y[j]; a.y[j] = u;
    u = a.k[i]; a.k[i] = a.k[j]; a.k[j] = u;
}

// Bitonic sort of P (a power of two) entries, best key first.  Every thread
// of the block takes part; the arrays may live in LDS or global memory.
__device__ void sort_best_first(const Keys& a, int P)
{
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                if (up ? kb(a, hi, lo) : kb(a, lo, hi)) kswap(a, lo, hi);
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ void set_sentinel(const Keys& a, int i)
{
    a.sw[i] = -INFINITY;
    a.s1[i] = -INFINITY;
    a.x[i] = 0x7fffffff;
    a.y[i] = 0x7fffffff;
    a.k[i] = 0x7fffffff;
}

__device__ __forceinline__ int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Greedy suppression over `a` sorted best first (N entries), run by wave 0:
// a pose is accepted iff its squared distance (scaled by 4^level) to every
// accepted pose is >= dmin2.  The distance test is exact: integer squared
// distance and a squared float, both exact in FP64.
__device__ int greedy_wave0(const Keys& a, int N, int level, double dmin2, int cap, int* ax, int* ay, int* aidx)
{
    const int lane = threadIdx.x & 63;
    int acc = 0;
    for (int c = 0; c < N && acc < cap; ++c) {
        const int x = a.x[c], y = a.y[c];
        bool sup = false;
        for (int q = lane; q < acc; q += 64) {
            const long long dx = (long long)x - ax[q], dy = (long long)y - ay[q];
            const long long d2 = (dx * dx + dy * dy) << (2 * level);
            sup |= (double)d2 < dmin2;
        }
        if (__ballot(sup) == 0ull) {
            if (lane == 0) {
                ax[acc] = x;
                ay[acc] = y;
                aidx[acc] = c;
            }
            __threadfence_block();
            ++acc;
        }
    }
    return acc;
}

constexpr int kSelCap = 2048;   // candidates sorted in LDS by k_select
constexpr int kFinCap = 1024;   // candidates handled by k_final

__global__ __launch_bounds__(1024) void k_select(const float* __restrict__ mw, const float* __restrict__ m1,
                                                  const int32_t* __restrict__ mk, int gw, int gh, int sx, int sy,
                                                  int level, float min_score, double dmin2, double theta_min,
                                                  double step_level, tm_pose* __restrict__ out, int cap,
                                                  int32_t* __restrict__ n_out, Keys g)
{
    __shared__ float l_sw[kSelCap], l_s1[kSelCap];
    __shared__ int l_x[kSelCap], l_y[kSelCap], l_k[kSelCap];
    __shared__ int acc_x[kFinCap], acc_y[kFinCap], acc_i[kFinCap];
    __shared__ int count, n_acc;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    const int np = gw * gh;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const float w = mw[p];
        if (!(w >= min_score)) continue;
        const int j = p / gw, i = p - j * gw;
        const float s = m1[p];
        bool is_max = true;
        for (int b = -1; b <= 1 && is_max; ++b) {
            for (int a = -1; a <= 1; ++a) {
                if (a == 0 && b == 0) continue;
                const int ii = i + a, jj = j + b;
                if (ii < 0 || ii >= gw || jj < 0 || jj >= gh) continue;
                const int q = jj * gw + ii;
                if (!key_better(w, s, i, j, 0, mw[q], m1[q], ii, jj, 0)) {
                    is_max = false;
                    break;
                }
            }
        }
        if (is_max) {
            const int idx = atomicAdd(&count, 1);
            g.sw[idx] = w;
            g.s1[idx] = s;
            g.x[idx] = i * sx;
            g.y[idx] = j * sy;
            g.k[idx] = mk[p];
        }
    }
    __syncthreads();
    const int N = count;
    const int P = next_pow2(N > 0 ? N : 1);
    Keys a;
    if (P <= kSelCap) {
        a = Keys{l_sw, l_s1, l_x, l_y, l_k};
        for (int i = threadIdx.x; i < P; i += blockDim.x) {
            if (i < N) {
                l_sw[i] = g.sw[i];
                l_s1[i] = g.s1[i];
                l_x[i] = g.x[i];
                l_y[i] = g.y[i];
                l_k[i] = g.k[i];
            } else {
                set_sentinel(a, i);
            }
        }
    } else {
        a = g;
        for (int i = N + threadIdx.x; i < P; i += blockDim.x) set_sentinel(a, i);
    }
    __syncthreads();
    sort_best_first(a, P);
    const int capc = cap < kFinCap ? cap : kFinCap;
    if (threadIdx.x < 64) {
        const int m = greedy_wave0(a, N, level, dmin2, capc, acc_x, acc_y, acc_i);
        if (threadIdx.x == 0) n_acc = m;
    }
    __syncthreads();
    const int m = n_acc;
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const int c = acc_i[t];
        tm_pose o;
        o.x = a.x[c];
        o.y = a.y[c];
        o.k = a.k[c];
        o.level = level;
        o.theta_deg = (float)level_theta(theta_min, step_level, a.k[c]);
        o.score_w = a.sw[c];
        o.score_1 = a.s1[c];
        o.reserved = 0;
        out[t] = o;
    }
    if (threadIdx.x == 0) *n_out = m;
}

__global__ __launch_bounds__(256) void k_final(const tm_pose* __restrict__ cand, const int32_t* __restrict__ n_cand,
                                                int max_cand, float min_score, double dmin2, double theta_min,
                                                double step0, tm_pose* __restrict__ out, int cap,
                                                int32_t* __restrict__ n_out)
{
    __shared__ float l_sw[kFinCap], l_s1[kFinCap];
    __shared__ int l_x[kFinCap], l_y[kFinCap], l_k[kFinCap], l_src[kFinCap];
    __shared__ int acc_x[kFinCap], acc_y[kFinCap], acc_i[kFinCap];
    __shared__ int count, n_acc;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    int nc = n_cand ? *n_cand : max_cand;
    nc = nc < max_cand ? nc : max_cand;
    nc = nc < kFinCap ? nc : kFinCap;
    for (int i = threadIdx.x; i < nc; i += blockDim.x) {
        const tm_pose c = cand[i];
        if (!(c.score_w >= min_score)) continue;
        const int idx = atomicAdd(&count, 1);
        l_sw[idx] = c.score_w;
        l_s1[idx] = c.score_1;
        l_x[idx] = c.x;
        l_y[idx] = c.y;
        l_k[idx] = c.k;
        l_src[idx] = i;
    }
    __syncthreads();
    const int N = count;
    const int P = next_pow2(N > 0 ? N : 1);
    Keys a{l_sw, l_s1, l_x, l_y, l_k};
    for (int i = N + threadIdx.x; i < P; i += blockDim.x) set_sentinel(a, i);
    __syncthreads();
    sort_best_first(a, P);
    if (threadIdx.x < 64) {
        const int m = greedy_wave0(a, N, 0, dmin2, cap < kFinCap ? cap : kFinCap, acc_x, acc_y, acc_i);
        if (threadIdx.x == 0) n_acc = m;
    }
    __syncthreads();
    const int m = n_acc;
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const int c = acc_i[t];
        tm_pose o;
        o.x = a.x[c];
        o.y = a.y[c];
        o.k = a.k[c];
        o.level = 0;
        o.score_w = a.sw[c];
        o.score_1 = a.s1[c];
        o.theta_deg = (float)level_theta(theta_min, step0, a.k[c]);
        o.reserved = 0;
        out[t] = o;
    }
    if (threadIdx.x == 0) *n_out = m;
}

}  // namespace

size_t select_workspace_bytes(int gw, int gh)
{
    size_t np = (size_t)gw * gh;
    size_t P = 1;
    while (P < np) P <<= 1;
    return P * 20 + 256;
}

hipError_t launch_select(const float* sw, const float* s1, const int32_t* k, int gw, int gh, int sx, int sy,
                         int level, float min_score, double dmin2, double theta_min, double step_level,
                         tm_pose* out, int capacity, int32_t* n_out, void* scratch, hipStream_t s)
{
    size_t np = (size_t)gw * gh;
    size_t P = 1;
    while (P < np) P <<= 1;
    Keys g;
    g.sw = reinterpret_cast<float*>(scratch);
    g.s1 = g.sw + P;
    g.x = reinterpret_cast<int*>(g.s1 + P);
    g.y = g.x + P;
    g.k = g.y + P;
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, sw, s1, k, gw, gh, sx, sy, level, min_score, dmin2,
                       theta_min, step_level, out, capacity, n_out, g);
    return hipGetLastError();
}

hipError_t launch_final(const tm_pose* cand, const int32_t* n_cand, int max_cand, float min_score, double dmin2,
                        double theta_min, double step0, tm_pose* out, int capacity, int32_t* n_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, cand, n_cand, max_cand, min_score, dmin2, theta_min, step0,
                       out, capacity, n_out);
    return hipGetLastError();
}

}  // namespace tmk
