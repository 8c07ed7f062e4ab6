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

__device__ __forceinline__ void kcopy(const Keys& dst, int i, const Keys& src, int j)
{
    dst.sw[i] = src.sw[j];
    dst.s1[i] = src.s1[j];
    dst.x[i] = src.x[j];
    dst.y[i] = src.y[j];
    dst.k[i] = src.k[j];
}

constexpr int kBuckets = 1024;

// S_w in [-1, 1] to a bucket, best first.  The map is monotone (1 - s is
// rounded monotonically, the scaling by 512 is exact), so a better S_w never
// lands in a later bucket and sorting each bucket by the full key sorts all.
__device__ __forceinline__ int score_bucket(float sw)
{
    const int b = (int)((1.0f - sw) * 512.0f);
    return b < 0 ? 0 : (b > kBuckets - 1 ? kBuckets - 1 : b);
}

// Exclusive prefix sum over the block (1024 threads, one value each).
__device__ int block_exclusive_scan(int v, int* wsum)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
        int t = lane < 16 ? wsum[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int u = __shfl_up(t, o, 64);
            if (lane >= o) t += u;
        }
        if (lane < 16) wsum[lane] = t;
    }
    __syncthreads();
    const int r = x - v + (w > 0 ? wsum[w - 1] : 0);
    __syncthreads();
    return r;
}

// Sort in[0..N) best first into out[0..N) (1024 threads): bucket by S_w, then
// each element's position inside its bucket is its rank by the full key
// among the bucket's members.  Positions are distinct, so ranks are too.
// cnt, off: kBuckets ints (LDS); idx: N ints; wsum: 16 ints.
__device__ void bucket_sort(const Keys& in, const Keys& out, int N, int* cnt, int* off, int* idx, int* wsum)
{
    cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) atomicAdd(&cnt[score_bucket(in.sw[i])], 1);
    __syncthreads();
    const int c = cnt[threadIdx.x];
    off[threadIdx.x] = block_exclusive_scan(c, wsum);
    cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int b = score_bucket(in.sw[i]);
        idx[off[b] + atomicAdd(&cnt[b], 1)] = i;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < N; s += blockDim.x) {
        const int i = idx[s];
        const int b = score_bucket(in.sw[i]);
        const int b0 = off[b], b1 = b0 + cnt[b];
        int rank = 0;
        for (int t = b0; t < b1; ++t) rank += kb(in, idx[t], i) ? 1 : 0;
        kcopy(out, b0 + rank, in, i);
    }
    __syncthreads();
}

// The squared distance d2 (scaled by 4^level) is an integer below 2^53 for
// any image this library accepts, so d2 < dmin2 exactly when d2 < lim with
// lim = ceil(dmin2) (dmin2 = dmin^2 is exact in FP64): the test runs in
// integers.
__device__ __forceinline__ long long dist_limit(double dmin2)
{
    return dmin2 >= 9.0e18 ? 0x7fffffffffffffffLL : (long long)ceil(dmin2);
}

__device__ __forceinline__ bool too_close(int x, int y, int ax, int ay, int level, long long lim)
{
    const long long dx = (long long)x - ax, dy = (long long)y - ay;
    const long long d2 = (dx * dx + dy * dy) << (2 * level);
    return d2 < lim;
}

// Greedy suppression over `a` sorted best first (N entries), run by wave 0:
// a pose is accepted iff its squared distance (scaled by 4^level) to every
// accepted pose is >= dmin2.  The distance test is exact (integers against
// dist_limit(dmin2)).  The wave takes 64
// candidates at a time: each lane tests its candidate against the poses
// accepted so far, then the survivors are accepted in key order, each one
// removing the later lanes it is too close to.
__device__ int greedy_wave0(const Keys& a, int N, int level, double dmin2, int cap, int* ax, int* ay, int* aidx)
{
    const int lane = threadIdx.x & 63;
    if (!(dmin2 > 0.0)) {
        // no squared distance is below a bound <= 0: the first poses are
        // accepted as they come
        const int m = N < cap ? N : cap;
        for (int c = lane; c < m; c += 64) {
            ax[c] = a.x[c];
            ay[c] = a.y[c];
            aidx[c] = c;
        }
        __threadfence_block();
        return m;
    }
    const long long lim = dist_limit(dmin2);
    int acc = 0;
    for (int c0 = 0; c0 < N && acc < cap; c0 += 64) {
        const int c = c0 + lane;
        const bool valid = c < N;
        const int x = valid ? a.x[c] : 0, y = valid ? a.y[c] : 0;
        bool sup = !valid;
        for (int q = 0; q < acc; ++q) sup |= too_close(x, y, ax[q], ay[q], level, lim);
        unsigned long long live = __ballot(!sup);
        while (live != 0ull && acc < cap) {
            const int j = __builtin_ctzll(live);  // wave-uniform: read the lane directly
            const int xj = __builtin_amdgcn_readlane(x, j), yj = __builtin_amdgcn_readlane(y, j);
            if (lane == 0) {
                ax[acc] = xj;
                ay[acc] = yj;
                aidx[acc] = c0 + j;
            }
            ++acc;
            live &= ~__ballot(too_close(x, y, xj, yj, level, lim));
            live &= (j == 63) ? 0ull : ~((2ull << j) - 1ull);
        }
        __threadfence_block();
    }
    return acc;
}

constexpr int kSelCap = 1024;   // candidates sorted into LDS by k_select (more go through global scratch)
constexpr int kFinCap = 1024;   // candidates handled by k_final

struct SelectArgs {
    int sx, sy, level, cap;
    float min_score;
    double theta_min, step_level;
    int K;  // angles of the level: map index m = j K + k (0: m is the angle index)
};

// One workgroup per pair (blockIdx.y).
__global__ __launch_bounds__(1024) void k_select(SelectArgs sa, const PairDesc* __restrict__ pairs)
{
    const PairDesc& P = pairs[blockIdx.y];
    const float* __restrict__ mw = P.mw;
    const float* __restrict__ m1 = P.m1;
    const int32_t* __restrict__ mk = P.mk;
    const int gw = P.gw, gh = P.gh, sx = sa.sx, sy = sa.sy, level = sa.level, cap = sa.cap;
    const float min_score = sa.min_score;
    const double dmin2 = (double)P.dmin * (double)P.dmin;
    const double theta_min = sa.theta_min, step_level = sa.step_level;
    tm_pose* __restrict__ out = P.cand;
    int32_t* __restrict__ n_out = P.ncand;
    const size_t npg = (size_t)gw * gh;
    Keys g{P.sel, P.sel + npg, reinterpret_cast<int*>(P.sel + 2 * npg), reinterpret_cast<int*>(P.sel + 3 * npg),
           reinterpret_cast<int*>(P.sel + 4 * npg)};
    Keys gs{P.sel + 5 * npg, P.sel + 6 * npg, reinterpret_cast<int*>(P.sel + 7 * npg),
            reinterpret_cast<int*>(P.sel + 8 * npg), reinterpret_cast<int*>(P.sel + 9 * npg)};
    int* gidx = reinterpret_cast<int*>(P.sel + 10 * npg);
    __shared__ float l_sw[kSelCap], l_s1[kSelCap];
    __shared__ int l_x[kSelCap], l_y[kSelCap], l_k[kSelCap];
    __shared__ int acc_x[kFinCap], acc_y[kFinCap], acc_i[kFinCap];
    __shared__ int cnt[kBuckets], off[kBuckets], wsum[16];
    __shared__ int count, n_acc;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    const int np = gw * gh;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const float w = mw[p];
        if (!(w >= min_score)) continue;  // most translations: below the floor, one load
        const int j = p / gw, i = p - j * gw;
        const float s = m1[p];
        // the 8 neighbours' S_w loaded at clamped addresses, then compared;
        // a neighbour's S_1 only decides (and is only read) on an equal S_w
        float nw[8];
        int nq[8];
        bool nin[8];
        int c = 0;
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
                if (a == 0 && b == 0) continue;
                const int ii = i + a, jj = j + b;
                nin[c] = (unsigned)ii < (unsigned)gw && (unsigned)jj < (unsigned)gh;
                nq[c] = min(max(jj, 0), gh - 1) * gw + min(max(ii, 0), gw - 1);
                nw[c] = mw[nq[c]];
                ++c;
            }
        }
        bool is_max = true;
        c = 0;
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
                if (a == 0 && b == 0) continue;
                if (nin[c] && !(nw[c] < w)) {  // otherwise this pose is strictly better
                    const float n1 = nw[c] == w ? m1[nq[c]] : 0.0f;
                    is_max = is_max && key_better(w, s, i, j, 0, nw[c], n1, i + a, j + b, 0);
                }
                ++c;
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
    Keys a;
    if (N <= kSelCap) {
        a = Keys{l_sw, l_s1, l_x, l_y, l_k};
        bucket_sort(g, a, N, cnt, off, acc_i, wsum);  // acc_i doubles as the index buffer
    } else {
        a = gs;
        bucket_sort(g, a, N, cnt, off, gidx, wsum);
    }
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
        const int mi = a.k[c];
        o.x = a.x[c];
        o.y = a.y[c];
        o.k = sa.K > 0 ? mi % sa.K : mi;
        o.j = sa.K > 0 ? mi / sa.K : 0;
        o.level = level;
        o.theta_deg = (float)level_theta(theta_min, step_level, o.k);
        o.score_w = a.sw[c];
        o.score_1 = a.s1[c];
        out[t] = o;
    }
    if (threadIdx.x == 0) *n_out = m;
}

// Final selection of the refined level-0 poses: score floor, key order (rank
// by counting, the list is short), greedy suppression, at most cap matches;
// the first min(matches, buf) are written and the count of matches, so a
// count above buf tells the caller that the result was truncated.
struct FinalArgs {
    int max_cand, cap;
    int buf;         // poses the result buffer holds
    float min_score;
    double theta_min, step0;
    int K0;  // angles of level 0; the key's last component is m = j K0 + k
    tm_pose* out;    // one pair: results here instead of at the pair's own buffers (null: the pair's)
    int32_t* n_out;
    int pick;        // >= 0: take each candidate as the best of its 27 level-0 sums (the refinement's
                     // last pick), centre from buffer ctr[pick]; < 0: candidates as they are
    int full;        // angle grid wraps (for the pick)
};

// One workgroup per pair (blockIdx.y).
__global__ __launch_bounds__(1024) void k_final(FinalArgs fa, const PairDesc* __restrict__ pairs)
{
    const PairDesc& P = pairs[blockIdx.y];
    const tm_pose* __restrict__ cand = P.cand;
    const int32_t* __restrict__ n_cand = P.ncand;
    const int max_cand = fa.max_cand, cap = fa.cap;
    const float min_score = fa.min_score;
    const double dmin2 = (double)P.dmin * (double)P.dmin;
    const double theta_min = fa.theta_min, step0 = fa.step0;
    tm_pose* __restrict__ out = fa.out ? fa.out : P.out;
    int32_t* __restrict__ n_out = fa.out ? fa.n_out : P.n_out;
    __shared__ float u_sw[kFinCap], u_s1[kFinCap];
    __shared__ int u_x[kFinCap], u_y[kFinCap], u_k[kFinCap];
    __shared__ float l_sw[kFinCap], l_s1[kFinCap];
    __shared__ int l_x[kFinCap], l_y[kFinCap], l_k[kFinCap];
    __shared__ int acc_x[kFinCap], acc_y[kFinCap], acc_i[kFinCap];
    __shared__ int count, n_acc;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    int nc = n_cand ? *n_cand : max_cand;
    nc = nc < max_cand ? nc : max_cand;
    nc = nc < kFinCap ? nc : kFinCap;
    if (fa.pick >= 0) {
        // one wave per candidate: the best of the 27 poses around its centre
        const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
        for (int i = wv; i < nc; i += nw) {
            const tm_pose ctr = P.ctr[fa.pick][i];
            float sw, s1;
            int x, y, k;
            pick27(P.part[0] + (size_t)i * kPartPerCand, ctr.x, ctr.y, ctr.k, P.W[0], P.H[0], P.n[0], fa.K0, fa.full, &sw, &s1,
                   &x, &y, &k);
            if ((threadIdx.x & 63) == 0 && sw >= min_score) {
                const int idx = atomicAdd(&count, 1);
                u_sw[idx] = sw;
                u_s1[idx] = s1;
                u_x[idx] = x;
                u_y[idx] = y;
                u_k[idx] = ctr.j * fa.K0 + k;
            }
        }
    } else {
        for (int i = threadIdx.x; i < nc; i += blockDim.x) {
            const tm_pose c = cand[i];
            if (!(c.score_w >= min_score)) continue;
            const int idx = atomicAdd(&count, 1);
            u_sw[idx] = c.score_w;
            u_s1[idx] = c.score_1;
            u_x[idx] = c.x;
            u_y[idx] = c.y;
            u_k[idx] = c.j * fa.K0 + c.k;
        }
    }
    __syncthreads();
    const int N = count;
    Keys u{u_sw, u_s1, u_x, u_y, u_k};
    Keys a{l_sw, l_s1, l_x, l_y, l_k};
    // duplicates (equal keys) keep their relative order by arrival index
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        int rank = 0;
        for (int j = 0; j < N; ++j) rank += (kb(u, j, i) || (j < i && !kb(u, i, j))) ? 1 : 0;
        kcopy(a, rank, u, i);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int m = greedy_wave0(a, N, 0, dmin2, cap < kFinCap ? cap : kFinCap, acc_x, acc_y, acc_i);
        if (threadIdx.x == 0) n_acc = m;
    }
    __syncthreads();
    const int m = n_acc;
    const int mw = m < fa.buf ? m : fa.buf;  // written: the best by key first
    for (int t = threadIdx.x; t < mw; t += blockDim.x) {
        const int c = acc_i[t];
        tm_pose o;
        const int mi = a.k[c];
        o.x = a.x[c];
        o.y = a.y[c];
        o.k = mi % fa.K0;
        o.j = mi / fa.K0;
        o.level = 0;
        o.score_w = a.sw[c];
        o.score_1 = a.s1[c];
        o.theta_deg = (float)level_theta(theta_min, step0, o.k);
        out[t] = o;
    }
    if (threadIdx.x == 0) *n_out = m;
}

}  // namespace

size_t select_scratch_bytes(int np) { return (size_t)np * 44 + 256; }

hipError_t launch_select(const SearchDesc& s, const PairDesc* d, int npairs, int max_np, hipStream_t st)
{
    (void)max_np;
    SelectArgs a;
    a.sx = s.sx;
    a.sy = s.sy;
    a.level = s.level;
    a.cap = s.max_cand;
    a.min_score = s.min_score;
    a.theta_min = s.theta_min;
    a.step_level = s.step[s.level];
    a.K = s.S > 1 ? s.K[s.level] : 0;
    hipLaunchKernelGGL(k_select, dim3(1, npairs), dim3(1024), 0, st, a, d);
    return hipGetLastError();
}

hipError_t launch_final(const SearchDesc& s, const PairDesc* d, int npairs, hipStream_t st, tm_pose* out,
                        int32_t* n_out, int pick)
{
    FinalArgs a;
    a.pick = pick;
    a.full = s.full;
    a.out = npairs == 1 ? out : nullptr;
    a.n_out = n_out;
    a.max_cand = s.max_cand;
    a.cap = s.max_matches;
    a.buf = s.capacity;
    a.min_score = s.min_score;
    a.theta_min = s.theta_min;
    a.step0 = s.step[0];
    a.K0 = s.K[0] > 0 ? s.K[0] : 1;
    hipLaunchKernelGGL(k_final, dim3(1, npairs), dim3(1024), 0, st, a, d);
    return hipGetLastError();
}

}  // namespace tmk
