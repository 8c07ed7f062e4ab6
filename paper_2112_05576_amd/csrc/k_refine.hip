// Coarse-to-fine refinement.  The paper starts the score computation at the
// top image of the pyramid (Sec. II para. 2); each candidate found there is
// carried down one level at a time by re-scoring the 27 poses
// (2x + a, 2y + b, 2k + c), a, b, c in {-1, 0, 1}, with the same windowed
// score (Eq. 1) and keeping the best by the selection key.
//
// One pass per level, by one of two kernels with the same arithmetic.  The
// points of a pose are shared by kThreads threads (thread t takes the points
// t, t + kThreads, ...), and the sums are kept per wave of them:
//  * k_refine_level, one workgroup of one wave per (candidate, angle, wave):
//    each lane forms q_i and r_i of its points in FP64, reads the 5x5 field
//    block covering the 3x3 windows of the 9 translations straight from
//    memory (two points' 50 loads in flight), and accumulates 9 windowed and
//    9 centre votes;
//  * k_refine_tile, one workgroup per candidate: the candidate's whole field
//    block (side 2 rad + 5 around (2x, 2y)) is first staged in LDS with
//    coalesced loads, then three groups of kThreads threads score the three
//    angles as above with the taps read from LDS.
// A thread adds its points in increasing order and each wave combines its
// lanes by a fixed butterfly, in both kernels, so their per-wave sums are
// bit-identical and a launch may take either; whoever picks from them adds
// the waves in order.  The gathers are bound by the address rate of each
// CU's vector memory unit (every lane's block lies elsewhere), so they are
// spread one wave per workgroup over as many CUs as the candidates allow;
// the staged kernel pays off once a launch holds many candidates.  The next
// level (or the final pick) picks the best of the 27 sums.
#include "tm_device.h"

namespace tmk {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
static_assert(kWaves == kRefineWaves, "sums are kept per wave of a pose's threads");
constexpr size_t kTileMax = 128 * 1024;  // largest staged field block

struct LevelArgs {
    int level;             // l, the level scored
    int pick;              // 1: pick the pose of level l+1 from its sums; 0: poses are given
    int K, K_above;        // angles of levels l and l+1
    double step, step_above;
    int full, win, max_cand;
    double theta_min;
    int src;               // centre buffer read (0/1); the other one is written
    int staged;            // pairs with rtile[level] set are refined by k_refine_tile
    double sigma_min, sigma_step;  // scale grid; a candidate keeps its scale index j
    int S;                         // scales (indices outside 0 .. S-1 are clamped)
};
// (the window reading, tm_vote, is the kernels' VOTE template argument)

// Field element (an FP32 pair), the rotated model direction in the form its
// product takes, and the product (FP32 products and sum).  The refinement
// always reads FP32 fields: an FP16 pyramid keeps an FP32 twin for it.
template <int PREC>
struct Raw;
template <>
struct Raw<TM_FP32> {
    using T = float2;
    using R = float2;
    static __device__ __forceinline__ T zero() { return make_float2(0.f, 0.f); }
    static __device__ __forceinline__ T load(const void* f, size_t o) { return reinterpret_cast<const float2*>(f)[o]; }
    static __device__ __forceinline__ R dir(double rx, double ry) { return make_float2((float)rx, (float)ry); }
    static __device__ __forceinline__ float dot(R r, T g) { return r.x * g.x + r.y * g.y; }
    static __device__ __forceinline__ bool edge(T g) { return g.x != 0.0f || g.y != 0.0f; }
};

// The 9 windowed votes and 9 centre votes of one point from the 5x5 block of
// field values around its projection (taps outside the image vote 0).  VOTE
// 1: the edge-taps-only window (off-edge and outside taps enter the maxima as
// kOffEdge, each maximum is finished by vote_finish); centre votes as in 0.
// ZEROS: the block already holds (+0, +0) outside the image (a staged tile),
// so no tap needs its position tested: such a tap's product is a zero of
// either sign, which changes no maximum but a zero's sign and no sum at all
// (every sum starts at +0, and x + (-0) = x), and it is off the edge set.
template <int PREC, int VOTE, bool ZEROS = false>
__device__ __forceinline__ void votes5x5(const typename Raw<PREC>::T (&gv)[5][5], const bool (&rin)[5],
                                         const bool (&cin)[5], typename Raw<PREC>::R r, float (&aw)[9], float (&a1)[9])
{
    float D[5][5], E[5][5];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            const float d = Raw<PREC>::dot(r, gv[v][u]);
            const bool in = ZEROS || (rin[v] && cin[u]);
            D[v][u] = in ? d : 0.0f;
            if constexpr (VOTE == 1)
                E[v][u] = (in && Raw<PREC>::edge(gv[v][u])) ? d : kOffEdge;
            else
                E[v][u] = D[v][u];
        }
    float hm[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int u = 0; u < 3; ++u) hm[v][u] = fmaxf(fmaxf(E[v][u], E[v][u + 1]), E[v][u + 2]);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            aw[b * 3 + u] += win_finish<VOTE>(fmaxf(fmaxf(hm[b][u], hm[b + 1][u]), hm[b + 2][u]));
            a1[b * 3 + u] += D[b + 1][u + 1];
        }
}

// One step of the reduce-scatter below: N slots (values base .. base + n - 1
// of the 18, n <= N, the rest padding) to H = (N + 1) / 2 slots.  The lane
// with the offset's bit clear keeps the first H slots and the other lane the
// rest; each kept slot adds the partner's slot of the same value.
template <int N>
__device__ __forceinline__ void rs_step(float (&v)[N], float (&k)[(N + 1) / 2], int off, int& base, int& n)
{
    constexpr int H = (N + 1) / 2;
    const bool hi = (threadIdx.x & off) != 0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const float lo_v = v[j], hi_v = H + j < N ? v[H + j] : 0.0f;
        const float keep = hi ? hi_v : lo_v, send = hi ? lo_v : hi_v;
        k[j] = keep + __shfl_xor(send, off, 64);
    }
    if (hi) {
        base += H;
        n -= H;
    } else if (n > H) {
        n = H;
    }
}

// The 18 sums of one wave, written to out[0..17].  The pairs added are those
// of the butterfly over lane offsets 32, 16, .., 1 (each partial is the sum
// of the same two operands, and addition commutes), so every sum has the
// bits of that butterfly's; the values are split between the lanes as they
// go (9, 5, 3, 2, 1 slots, then one pair), 21 shuffles instead of 108, and
// the lane that ends with a value writes it.
__device__ __forceinline__ void wave_sum18(float (&aw)[9], float (&a1)[9], float* out)
{
    float v18[18];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        v18[m] = aw[m];
        v18[9 + m] = a1[m];
    }
    int base = 0, n = 18;
    float v9[9], v5[5], v3[3], v2[2], v1[1];
    rs_step<18>(v18, v9, 32, base, n);
    rs_step<9>(v9, v5, 16, base, n);
    rs_step<5>(v5, v3, 8, base, n);
    rs_step<3>(v3, v2, 4, base, n);
    rs_step<2>(v2, v1, 2, base, n);
    const float s = v1[0] + __shfl_xor(v1[0], 1, 64);
    if ((threadIdx.x & 1) == 0 && n > 0) out[base] = s;
}

// The candidate's pose at the level above: picked by the first wave from that
// level's sums (or the candidate itself on the first refined level),
// published in cur[0..3] (x, y, angle index, scale index); `writer` also
// records it as the centre.  The 27 poses of a pick share the scale, so the
// key's last component (the pose index j K + k) orders them as k does.  c <
// max_cand, whose slots every buffer holds, so the reads are taken before the
// candidate count is known (their latencies overlap) and only `live` (c below
// the count) lets the results out.
__device__ void take_centre(const LevelArgs& a, const PairDesc& P, int c, bool writer, bool live, int* cur)
{
    const int l = a.level;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        int x, y, k, j;
        float sw, s1;
        if (a.pick) {
            const tm_pose ctr = P.ctr[a.src][c];
            const int la = l + 1;
            pick27(P.part[la] + (size_t)c * kPartPerCand, ctr.x, ctr.y, ctr.k, P.W[la], P.H[la], P.n[la], a.K_above,
                   a.full, &sw, &s1, &x, &y, &k);
            j = ctr.j;
        } else {
            const tm_pose p = P.cand[c];
            x = p.x;
            y = p.y;
            k = p.k;
            j = p.j;
            sw = p.score_w;
            s1 = p.score_1;
        }
        j = min(max(j, 0), a.S - 1);  // poses given by a caller may name any scale
        if (lane == 0 && live) {
            cur[0] = x;
            cur[1] = y;
            cur[2] = k;
            cur[3] = j;
            if (writer) {
                tm_pose o;
                o.x = x;
                o.y = y;
                o.k = k;
                o.level = l + 1;
                o.theta_deg = (float)level_theta(a.theta_min, a.step_above, k);
                o.score_w = sw;
                o.score_1 = s1;
                o.j = j;
                P.ctr[a.src ^ 1][c] = o;
            }
        }
    }
}

// Block geometry of one point at (px, py): in-image rows and columns of the
// 5x5 block, clamped column indices and row offsets.
struct Block5 {
    bool rin[5], cin[5];
    int col[5];
    size_t rowoff[5];
};

__device__ __forceinline__ void block5(int px, int py, int W, int H, Block5& b)
{
#pragma unroll
    for (int u = 0; u < 5; ++u) {
        const int xx = px - 2 + u, yy = py - 2 + u;
        b.cin[u] = (unsigned)xx < (unsigned)W;
        b.rin[u] = (unsigned)yy < (unsigned)H;
        b.col[u] = min(max(xx, 0), W - 1);
        b.rowoff[u] = (size_t)min(max(yy, 0), H - 1) * W;
    }
}

// The 9 windowed and 9 centre votes of the points t, t + kThreads, ... of
// level l for the pose (2x + ., 2y + ., angle with cosine/sine cs, sn, scale
// sigma), added to aw / a1 in point order; field taps gathered from memory.
template <int PREC, int VOTE>
__device__ __forceinline__ void gather_votes(const PairDesc& P, int l, int win, int x, int y, double cs, double sn,
                                             double sigma, int t, float (&aw)[9], float (&a1)[9])
{
    const void* field = P.field[l];
    const int W = P.W[l], H = P.H[l], n = P.n[l];
    const ModelPoint* __restrict__ pts = P.pts[l];
    const double2* __restrict__ dir = P.dir[l];
    const int wh = (win - 1) / 2;
    if (wh == 1) {
        // two points per step (this thread's next two), their 50 loads issued
        // before any is used; votes added in point order
        for (int i = t; i < n; i += 2 * kThreads) {
            const int j = i + kThreads;
            const bool two = j < n;
            int qx0, qy0, qx1 = 0, qy1 = 0;
            double rx0, ry0, rx1 = 0, ry1 = 0;
            const double2 d0 = dir[i], d1 = dir[two ? j : i];
            project_dir_s(pts[i], d0.x, d0.y, cs, sn, sigma, &qx0, &qy0, &rx0, &ry0);
            if (two) project_dir_s(pts[j], d1.x, d1.y, cs, sn, sigma, &qx1, &qy1, &rx1, &ry1);
            Block5 b0, b1;
            block5(2 * x + qx0, 2 * y + qy0, W, H, b0);
            block5(2 * x + qx1, 2 * y + qy1, W, H, b1);
            typename Raw<PREC>::T g0[5][5], g1[5][5];
#pragma unroll
            for (int v = 0; v < 5; ++v)
#pragma unroll
                for (int u = 0; u < 5; ++u) {
                    g0[v][u] = Raw<PREC>::load(field, b0.rowoff[v] + b0.col[u]);
                    g1[v][u] = Raw<PREC>::load(field, b1.rowoff[v] + b1.col[u]);
                }
            __builtin_amdgcn_sched_barrier(0);
            votes5x5<PREC, VOTE>(g0, b0.rin, b0.cin, Raw<PREC>::dir(rx0, ry0), aw, a1);
            if (two) votes5x5<PREC, VOTE>(g1, b1.rin, b1.cin, Raw<PREC>::dir(rx1, ry1), aw, a1);
        }
    } else {
        // any odd window: direct evaluation of each translation
        for (int i = t; i < n; i += kThreads) {
            int qx, qy;
            double rx, ry;
            const double2 d = dir[i];
            project_dir_s(pts[i], d.x, d.y, cs, sn, sigma, &qx, &qy, &rx, &ry);
            const float fx = (float)rx, fy = (float)ry;
            const int px = 2 * x + qx, py = 2 * y + qy;
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    const int cx = px + u - 1, cy = py + b - 1;
                    float best = -INFINITY;
                    for (int dy = -wh; dy <= wh; ++dy)
                        for (int dx = -wh; dx <= wh; ++dx)
                            best = fmaxf(best, field_win_tap<PREC, VOTE>(field, W, H, cx + dx, cy + dy, fx, fy));
                    aw[b * 3 + u] += win_finish<VOTE>(best);
                    a1[b * 3 + u] += field_dot<PREC>(field, W, H, cx, cy, fx, fy);
                }
        }
    }
}

template <int PREC, int VOTE>
__global__ __launch_bounds__(64) void k_refine_level(LevelArgs a, const PairDesc* __restrict__ pairs)
{
    __shared__ int cur[4];
    const PairDesc& P = pairs[blockIdx.y];
    const int l = a.level;
    if (a.staged && P.rtile[l]) return;  // this pair's level is refined by k_refine_tile
    const int c = blockIdx.x / (3 * kWaves);
    const int g = blockIdx.x / kWaves % 3, w = blockIdx.x % kWaves;
    const int count = P.ncand ? min(a.max_cand, *P.ncand) : a.max_cand;
    take_centre(a, P, c, g == 0 && w == 0, c < count, cur);
    if (c >= count) return;
    __syncthreads();
    const int x = cur[0], y = cur[1], k = cur[2];
    const double sigma = scale_of(a.sigma_min, a.sigma_step, cur[3]);
    const int kc = angle_index(2 * k + g - 1, a.K, a.full);
    double cs, sn;
    sincos_deg(level_theta(a.theta_min, a.step, kc), &cs, &sn);
    float aw[9], a1[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        aw[m] = 0.f;
        a1[m] = 0.f;
    }
    gather_votes<PREC, VOTE>(P, l, a.win, x, y, cs, sn, sigma, w * 64 + (int)threadIdx.x, aw, a1);
    wave_sum18(aw, a1, P.part[l] + (size_t)c * kPartPerCand + (g * kWaves + w) * 18);
}

// One workgroup per candidate, three groups of kThreads threads, group g
// scoring angle 2k + g - 1 from the one staged block: thread t of a group
// takes the points t, t + kThreads, ... as a thread of k_refine_level does,
// and each group reduces as one of its workgroups, so the sums are the same
// bits.  Three times the waves of one group share the block's LDS.
constexpr int kTileGroups = 3;

template <int PREC, int VOTE>
__global__ __launch_bounds__(kThreads * kTileGroups) void k_refine_tile(LevelArgs a, const PairDesc* __restrict__ pairs)
{
    using T = typename Raw<PREC>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cur[4];
    // an image's candidates run on one XCD, whose L2 then serves their
    // overlapping blocks
    const uint3 B = xcd_block();  // (candidate, pair)
    const PairDesc& P = pairs[B.y];
    const int l = a.level;
    if (!P.rtile[l]) return;
    const int c = B.x;
    const int count = P.ncand ? min(a.max_cand, *P.ncand) : a.max_cand;
    take_centre(a, P, c, true, c < count, cur);
    if (c >= count) return;
    __syncthreads();
    const int x = cur[0], y = cur[1], k = cur[2];
    const double sigma = scale_of(a.sigma_min, a.sigma_step, cur[3]);
    const void* field = P.field[l];
    const int W = P.W[l], H = P.H[l], n = P.n[l];
    const ModelPoint* __restrict__ pts = P.pts[l];
    const double2* __restrict__ dir = P.dir[l];
    const int rad = P.rad_l[l];
    const int S = 2 * rad + 5, SS = S * S;
    const int ox = 2 * x - rad - 2, oy = 2 * y - rad - 2;
    T* tile = reinterpret_cast<T*>(smem);
    // stage: 8 loads in flight per thread (clamped addresses, zero selected
    // outside the image)
    constexpr int kU = 8, kAll = kThreads * kTileGroups;
    for (int e0 = threadIdx.x; e0 < SS; e0 += kU * kAll) {
        T v[kU];
        bool ok[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const int e = min(e0 + j * kAll, SS - 1);
            const int r = e / S, cc = e - r * S;
            const int gx = ox + cc, gy = oy + r;
            ok[j] = (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H;
            v[j] = Raw<PREC>::load(field, (size_t)min(max(gy, 0), H - 1) * W + min(max(gx, 0), W - 1));
        }
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const int e = e0 + j * kAll;
            if (e < SS) tile[e] = ok[j] ? v[j] : Raw<PREC>::zero();
        }
    }
    __syncthreads();
    {
        const int g = threadIdx.x / kThreads, t = threadIdx.x - g * kThreads;
        const int kc = angle_index(2 * k + g - 1, a.K, a.full);
        double cs, sn;
        sincos_deg(level_theta(a.theta_min, a.step, kc), &cs, &sn);
        float aw[9], a1[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) {
            aw[m] = 0.f;
            a1[m] = 0.f;
        }
        for (int i = t; i < n; i += kThreads) {
            int qx, qy;
            double rx, ry;
            const double2 d = dir[i];
            project_dir_s(pts[i], d.x, d.y, cs, sn, sigma, &qx, &qy, &rx, &ry);
            const int px = 2 * x + qx, py = 2 * y + qy;
            // |q| < rad per component, so the block covers px - 2 .. px + 2
            const T* b = tile + (size_t)(py - 2 - oy) * S + (px - 2 - ox);
            // the staged block is zero outside the image: no tap is tested
            const bool none[5] = {};
            T gv[5][5];
#pragma unroll
            for (int v = 0; v < 5; ++v)
#pragma unroll
                for (int u = 0; u < 5; ++u) gv[v][u] = b[v * S + u];
            votes5x5<PREC, VOTE, true>(gv, none, none, Raw<PREC>::dir(rx, ry), aw, a1);
        }
        wave_sum18(aw, a1, P.part[l] + (size_t)c * kPartPerCand + (g * kWaves + (t >> 6)) * 18);
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
    pick27(P.part[0] + (size_t)c * kPartPerCand, ctr.x, ctr.y, ctr.k, P.W[0], P.H[0], P.n[0], a.K0, a.full, &sw, &s1, &x, &y,
           &k);
    if (threadIdx.x == 0) {
        tm_pose o;
        o.x = x;
        o.y = y;
        o.k = k;
        o.level = 0;
        o.theta_deg = (float)level_theta(a.theta_min, a.step0, k);
        o.score_w = sw;
        o.score_1 = s1;
        o.j = ctr.j;  // written by take_centre, already in range
        P.cand[c] = o;
    }
}

}  // namespace

size_t refine_tile_bytes(int rad, int precision)
{
    const size_t S = 2 * (size_t)rad + 5;
    return S * S * (precision == TM_FP16 ? 4 : 8);
}

bool refine_tile_fits(int rad, int precision, int win)
{
    return win == 3 && refine_tile_bytes(rad, precision) <= kTileMax;
}

hipError_t prepare_refine()
{
    static bool done = false;
    if (done) return hipSuccess;
    const void* k[] = {reinterpret_cast<const void*>(&k_refine_tile<TM_FP32, 0>),
                       reinterpret_cast<const void*>(&k_refine_tile<TM_FP32, 1>)};
    for (const void* f : k) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileMax);
        if (e != hipSuccess) return e;
    }
    done = true;
    return hipSuccess;
}

namespace {
template <int VOTE>
void launch_level_kernels(const SearchDesc& s, const PairDesc* d, int npairs, const RefinePlan& rp, int l,
                          const LevelArgs& a, hipStream_t st)
{
    // the descriptors' fields are FP32 (an FP16 pyramid's twin): the
    // refinement's picks are decisions, taken at FP32 accuracy
    if (!rp.staged || rp.gather[l]) {
        dim3 grid((unsigned)(s.max_cand * 3 * kWaves), npairs);
        hipLaunchKernelGGL((k_refine_level<TM_FP32, VOTE>), grid, dim3(64), 0, st, a, d);
    }
    if (rp.staged && rp.tile_bytes[l] > 0) {
        dim3 grid((unsigned)s.max_cand, npairs);
        hipLaunchKernelGGL((k_refine_tile<TM_FP32, VOTE>), grid, dim3(kThreads * kTileGroups), rp.tile_bytes[l], st,
                           a, d);
    }
}
}  // namespace

hipError_t launch_refine(const SearchDesc& s, const PairDesc* d, int npairs, int from_level, const RefinePlan& rp,
                         hipStream_t st, bool pick)
{
    if (from_level <= 0 || npairs == 0) return hipSuccess;
    from_level = min(from_level, s.L - 1);
    hipError_t e = prepare_refine();
    if (e != hipSuccess) return e;
    int src = 0;
    for (int l = from_level - 1; l >= 0; --l) {
        LevelArgs a;
        a.level = l;
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
        a.staged = rp.staged;
        a.sigma_min = s.sigma_min;
        a.sigma_step = s.sigma_step;
        a.S = s.S > 0 ? s.S : 1;
        if (s.vote)
            launch_level_kernels<1>(s, d, npairs, rp, l, a, st);
        else
            launch_level_kernels<0>(s, d, npairs, rp, l, a, st);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        src ^= 1;
    }
    if (!pick) return hipSuccess;  // the final selection picks (launch_final with the centre buffer)
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
