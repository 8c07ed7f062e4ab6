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

// Sort in[0..N) best first into out[0..N) by counting, for N <= 1024 (1024
// threads): G lanes of one wave share a pose i (G the largest power of two
// up to 64 with G N <= 1024), each counts the poses better than i among every
// G-th one, and the G counts are added across the lanes.  With ties (equal
// keys), the earlier one in `in` goes first.
template <bool TIES>
__device__ void rank_sort(const Keys& in, const Keys& out, int N)
{
    int G = 64;
    while (G > 1 && G * N > (int)blockDim.x) G >>= 1;
    const int i = threadIdx.x / G, r = threadIdx.x & (G - 1);
    int c = 0;
    if (i < N) {
        const float w = in.sw[i], s = in.s1[i];
        const int x = in.x[i], y = in.y[i], k = in.k[i];
        for (int j = r; j < N; j += G) {
            const float jw = in.sw[j], js = in.s1[j];
            const int jx = in.x[j], jy = in.y[j], jk = in.k[j];
            bool b = key_better(jw, js, jx, jy, jk, w, s, x, y, k);
            if (TIES) b = b || (j < i && !key_better(w, s, x, y, k, jw, js, jx, jy, jk));
            c += b ? 1 : 0;
        }
    }
    for (int o = 1; o < G; o <<= 1) c += __shfl_xor(c, o, 64);
    if (i < N && r == 0) kcopy(out, c, in, i);
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

// Coordinates in [0, 2^15): d2 = dx^2 + dy^2 < 2^31 in 32-bit integers (the
// products in the 24-bit multiplier), tested against the limit divided by
// 4^level and rounded up: for an integer d2, d2 4^level < lim exactly when
// d2 < ceil(lim / 4^level).  Otherwise in 64 bits.
constexpr int kSmallCoord = 1 << 15;

__device__ __forceinline__ unsigned small_limit(long long lim, int level)
{
    const int s = 2 * level;
    const long long q = (lim >> s) + ((lim & ((1LL << s) - 1)) != 0 ? 1 : 0);
    return q > 0xffffffffLL ? 0xffffffffu : (unsigned)q;
}

template <bool SMALL>
__device__ __forceinline__ bool too_close(int x, int y, int ax, int ay, int level, long long lim, unsigned lim32)
{
    if (SMALL) {
        const int dx = x - ax, dy = y - ay;
        return (unsigned)(__mul24(dx, dx) + __mul24(dy, dy)) < lim32;
    }
    const long long dx = (long long)x - ax, dy = (long long)y - ay;
    const long long d2 = (dx * dx + dy * dy) << (2 * level);
    return d2 < lim;
}

// One chunk of up to 64 candidates at a time: every wave builds rows of the
// chunk's closeness matrix (row j: the lanes within the distance of lane j's
// pose, one ballot), wave 0 drops the lanes close to a pose accepted in an
// earlier chunk, then accepts the rest in rounds and writes the accepted
// poses in parallel.  A round accepts every live lane with no live lane
// before it in its row: the lanes before it that left the live set were each
// close to an accepted lane, so none of them is accepted, and the greedy pass
// in key order accepts it too; the accepted lanes and the lanes in their rows
// then leave the live set.  The first live lane is accepted in every round,
// so the rounds end, and they accept what the pass in key order accepts.  At
// most cap poses: the first ones of the accepted lanes, in lane order.
template <bool SMALL>
__device__ int greedy_run(const Keys& a, int N, int level, long long lim, int cap, int* ax, int* ay, int* aidx,
                          unsigned* rows, int* n_acc)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    const unsigned lim32 = SMALL ? small_limit(lim, level) : 0u;
    int acc = 0;
    for (int c0 = 0; c0 < N && acc < cap; c0 += 64) {
        const int nch = N - c0 < 64 ? N - c0 : 64;
        const bool valid = lane < nch;
        const int x = valid ? a.x[c0 + lane] : 0, y = valid ? a.y[c0 + lane] : 0;
        for (int j = wv; j < nch; j += nwv) {
            const int xj = a.x[c0 + j], yj = a.y[c0 + j];
            const unsigned long long m = __ballot(valid && too_close<SMALL>(x, y, xj, yj, level, lim, lim32));
            if (lane == 0) {
                rows[2 * j] = (unsigned)m;
                rows[2 * j + 1] = (unsigned)(m >> 32);
            }
        }
        bool sup = !valid;
        if (wv == 0)
            for (int q = 0; q < acc; ++q) sup |= too_close<SMALL>(x, y, ax[q], ay[q], level, lim, lim32);
        __syncthreads();
        if (wv == 0) {
            // a lane past the chunk is never live, so its stale row plays no part
            const unsigned long long row = ((unsigned long long)rows[2 * lane + 1] << 32) | rows[2 * lane];
            const unsigned long long before = (1ull << lane) - 1ull;
            unsigned long long live = __ballot(!sup), accm = 0ull;
            while (live != 0ull) {
                const unsigned long long f = __ballot(((live >> lane) & 1ull) && (row & live & before) == 0ull);
                accm |= f;
                live &= ~(f | __ballot((row & f) != 0ull));
            }
            const int room = cap - acc;
            const int pos = __popcll(accm & before);
            if (((accm >> lane) & 1ull) && pos < room) {
                ax[acc + pos] = x;
                ay[acc + pos] = y;
                aidx[acc + pos] = c0 + lane;
            }
            if (lane == 0) *n_acc = acc + min(__popcll(accm), room);
        }
        __syncthreads();
        acc = *n_acc;
    }
    return acc;
}

// Greedy suppression over `a` sorted best first (N entries), by the whole
// workgroup: a pose is accepted iff its squared distance (scaled by 4^level)
// to every accepted pose is >= dmin2, at most cap poses.  The distance test
// is exact (integers against dist_limit(dmin2)); `small`: every coordinate in
// [0, kSmallCoord).  Returns the count to every thread, with ax, ay (the
// accepted coordinates) and aidx (their places in `a`) written and visible.
// rows: 128 words of LDS; n_acc: one.
__device__ int greedy(const Keys& a, int N, int level, double dmin2, int cap, bool small, int* ax, int* ay,
                      int* aidx, unsigned* rows, int* n_acc)
{
    if (!(dmin2 > 0.0)) {
        // no squared distance is below a bound <= 0: the first poses are
        // accepted as they come
        const int m = N < cap ? N : cap;
        for (int c = threadIdx.x; c < m; c += blockDim.x) {
            ax[c] = a.x[c];
            ay[c] = a.y[c];
            aidx[c] = c;
        }
        __syncthreads();
        return m;
    }
    const long long lim = dist_limit(dmin2);
    return small ? greedy_run<true>(a, N, level, lim, cap, ax, ay, aidx, rows, n_acc)
                 : greedy_run<false>(a, N, level, lim, cap, ax, ay, aidx, rows, n_acc);
}

constexpr int kSelCap = 1024;   // candidates sorted into LDS by k_select (more go through global scratch)
constexpr int kFinCap = 1024;   // candidates handled by k_final
// bordered map cells whose S_w and S_1 k_select stages in LDS for the scan
// (an 80x60 grid takes 82x62 = 5084); with it the kernel holds about 73 KB of
// LDS, so two workgroups (pairs) share a CU
constexpr int kMapCap = 5120;
constexpr int kRankMax = 128;   // k_select sorts up to this many candidates by counting, more by buckets

// The strict local maxima of the key over the 8 neighbours on the translation
// grid, at or above the floor, in any order: appended to g and (the first
// kSelCap) to u.  W, S1: the best-angle S_w and S_1 maps (in LDS or global).
__device__ __forceinline__ void scan_maxima(const float* W, const float* S1, const int32_t* __restrict__ mk, int gw,
                                            int gh, int sx, int sy, float min_score, const Keys& g, const Keys& u,
                                            int* count)
{
    const int np = gw * gh;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const float w = W[p];
        if (!(w >= min_score)) continue;  // most translations: below the floor, one load
        const int j = p / gw, i = p - j * gw;
        const float s = S1[p];
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
                nw[c] = W[nq[c]];
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
                    const float n1 = nw[c] == w ? S1[nq[c]] : 0.0f;
                    is_max = is_max && key_better(w, s, i, j, 0, nw[c], n1, i + a, j + b, 0);
                }
                ++c;
            }
        }
        if (is_max) {
            const int idx = atomicAdd(count, 1);
            const int x = i * sx, y = j * sy, k = mk[p];
            g.sw[idx] = w;
            g.s1[idx] = s;
            g.x[idx] = x;
            g.y[idx] = y;
            g.k[idx] = k;
            if (idx < kSelCap) {
                u.sw[idx] = w;
                u.s1[idx] = s;
                u.x[idx] = x;
                u.y[idx] = y;
                u.k[idx] = k;
            }
        }
    }
}

// The same maxima from maps staged in LDS with a border of one cell (row
// pitch gw + 2, border S_w = -inf), one pass over the translations in steps of
// the workgroup size (row and column carried, no division).  Of the eight
// stored neighbours: one strictly above the pose makes it no maximum (it lies
// inside the grid, the border being -inf); all strictly below make it one
// (every neighbour inside the grid is below it, and only those count); any
// other pose (an equal S_w, a NaN) takes the tie rules above.
__device__ __forceinline__ void scan_maxima_staged(const float* W, const float* S1, const int32_t* __restrict__ mk,
                                                   int gw, int gh, int sx, int sy, float min_score, const Keys& g,
                                                   const Keys& u, int* count)
{
    const int np = gw * gh, pw = gw + 2, step = blockDim.x, dj = step / gw, di = step - dj * gw;
    int j = threadIdx.x / gw, i = threadIdx.x - j * gw;
    for (int p = threadIdx.x; p < np; p += step) {
        const int q = (j + 1) * pw + i + 1;
        const float w = W[q];
        if (w >= min_score) {
            const float nw[8] = {W[q - pw - 1], W[q - pw], W[q - pw + 1], W[q - 1],
                                 W[q + 1],      W[q + pw - 1], W[q + pw], W[q + pw + 1]};
            bool lower = true, higher = false;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                lower = lower && nw[c] < w;
                higher = higher || nw[c] > w;
            }
            bool is_max = !higher;
            if (!higher && !lower) {
                const float s = S1[q];
                int c = 0;
#pragma unroll
                for (int b = -1; b <= 1; ++b) {
#pragma unroll
                    for (int a = -1; a <= 1; ++a) {
                        if (a == 0 && b == 0) continue;
                        const bool nin = (unsigned)(i + a) < (unsigned)gw && (unsigned)(j + b) < (unsigned)gh;
                        if (nin && !(nw[c] < w)) {
                            const float n1 = nw[c] == w ? S1[q + b * pw + a] : 0.0f;
                            is_max = is_max && key_better(w, s, i, j, 0, nw[c], n1, i + a, j + b, 0);
                        }
                        ++c;
                    }
                }
            }
            if (is_max) {
                const int idx = atomicAdd(count, 1);
                const float s = S1[q];
                const int x = i * sx, y = j * sy, k = mk[p];
                g.sw[idx] = w;
                g.s1[idx] = s;
                g.x[idx] = x;
                g.y[idx] = y;
                g.k[idx] = k;
                if (idx < kSelCap) {
                    u.sw[idx] = w;
                    u.s1[idx] = s;
                    u.x[idx] = x;
                    u.y[idx] = y;
                    u.k[idx] = k;
                }
            }
        }
        i += di;
        j += dj;
        if (i >= gw) {
            i -= gw;
            ++j;
        }
    }
}

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
    // the maps staged for the scan; after it, the sorted keys and the bucket counters
    __shared__ int stage[2 * kMapCap];
    static_assert(5 * kSelCap + 2 * kBuckets + 128 <= 2 * kMapCap, "sort buffers exceed the map stage");
    __shared__ float u_sw[kSelCap], u_s1[kSelCap];
    __shared__ int u_x[kSelCap], u_y[kSelCap], u_k[kSelCap];
    __shared__ int acc_x[kFinCap], acc_y[kFinCap], acc_i[kFinCap];
    __shared__ int wsum[16];
    __shared__ int count, n_acc;
    if (threadIdx.x == 0) count = 0;
    const int np = gw * gh;
    const Keys u{u_sw, u_s1, u_x, u_y, u_k};
    const int pw = gw + 2;
    if ((long long)pw * (gh + 2) <= kMapCap) {
        // the maps into LDS with their border (four loads of each in flight
        // per thread), then the scan from LDS
        float* s_w = reinterpret_cast<float*>(stage);
        float* s_1 = s_w + kMapCap;
        for (int e = threadIdx.x; e < 2 * pw + 2 * gh; e += blockDim.x) {
            const int cell = e < pw ? e
                             : e < 2 * pw ? (gh + 1) * pw + (e - pw)
                             : e < 2 * pw + gh ? (e - 2 * pw + 1) * pw
                                               : (e - 2 * pw - gh + 1) * pw + pw - 1;
            s_w[cell] = -INFINITY;
            s_1[cell] = -INFINITY;
        }
        const int step = blockDim.x, dj = step / gw, di = step - dj * gw;
        int j = threadIdx.x / gw, i = threadIdx.x - j * gw;
        for (int p0 = 0; p0 < np; p0 += 4 * step) {
            float vw[4], v1[4];
            int dst[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = p0 + q * step + (int)threadIdx.x;
                vw[q] = p < np ? mw[p] : 0.0f;
                v1[q] = p < np ? m1[p] : 0.0f;
                dst[q] = (j + 1) * pw + i + 1;
                i += di;
                j += dj;
                if (i >= gw) {
                    i -= gw;
                    ++j;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = p0 + q * step + (int)threadIdx.x;
                if (p < np) {
                    s_w[dst[q]] = vw[q];
                    s_1[dst[q]] = v1[q];
                }
            }
        }
        __syncthreads();
        scan_maxima_staged(s_w, s_1, mk, gw, gh, sx, sy, min_score, g, u, &count);
    } else {
        __syncthreads();
        scan_maxima(mw, m1, mk, gw, gh, sx, sy, min_score, g, u, &count);
    }
    __syncthreads();
    const int N = count;
    int* cnt = stage + 5 * kSelCap;
    int* off = cnt + kBuckets;
    Keys a;
    if (N <= kSelCap) {
        a = Keys{reinterpret_cast<float*>(stage), reinterpret_cast<float*>(stage) + kSelCap, stage + 2 * kSelCap,
                 stage + 3 * kSelCap, stage + 4 * kSelCap};
        if (N <= kRankMax)
            rank_sort<false>(u, a, N);  // keys are distinct: (x, y) differ
        else
            bucket_sort(u, a, N, cnt, off, acc_i, wsum);  // acc_i doubles as the index buffer
    } else {
        a = gs;
        bucket_sort(g, a, N, cnt, off, gidx, wsum);
    }
    const int capc = cap < kFinCap ? cap : kFinCap;
    // x < gw sx and y < gh sy
    const bool small = (long long)gw * sx <= kSmallCoord && (long long)gh * sy <= kSmallCoord;
    const int m = greedy(a, N, level, dmin2, capc, small, acc_x, acc_y, acc_i,
                         reinterpret_cast<unsigned*>(off + kBuckets), &n_acc);
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
    __shared__ unsigned rows[128];
    __shared__ int count, n_acc, large;
    if (threadIdx.x == 0) {
        count = 0;
        large = 0;
    }
    __syncthreads();
    int nc = n_cand ? *n_cand : max_cand;
    nc = nc < max_cand ? nc : max_cand;
    nc = nc < kFinCap ? nc : kFinCap;
    if (fa.pick >= 0) {
        // half a wave per candidate: the best of the 27 poses around its centre
        const int h = threadIdx.x >> 5, nh = blockDim.x >> 5;
        for (int i0 = h & ~1; i0 < nc; i0 += nh) {  // both halves of a wave take the shuffles
            const int i = (i0 | (h & 1)) < nc ? (i0 | (h & 1)) : i0;
            const tm_pose ctr = P.ctr[fa.pick][i];
            float sw, s1;
            int x, y, k;
            pick27<32>(P.part[0] + (size_t)i * kPartPerCand, ctr.x, ctr.y, ctr.k, P.W[0], P.H[0], P.n[0], fa.K0, fa.full,
                       &sw, &s1, &x, &y, &k);
            if ((threadIdx.x & 31) == 0 && i == (i0 | (h & 1)) && sw >= min_score) {
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
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        if ((unsigned)u_x[i] >= (unsigned)kSmallCoord || (unsigned)u_y[i] >= (unsigned)kSmallCoord) large = 1;
    rank_sort<true>(u, a, N);  // duplicates (equal keys) keep their relative order by arrival index
    const int m = greedy(a, N, 0, dmin2, cap < kFinCap ? cap : kFinCap, large == 0, acc_x, acc_y, acc_i, rows, &n_acc);
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
