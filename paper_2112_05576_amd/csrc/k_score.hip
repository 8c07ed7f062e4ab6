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
// Every launch covers all (image, model) pairs of a batch: blockIdx.y (or z)
// is the pair.
#include <stdlib.h>

#include <algorithm>
#include <type_traits>

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

// max(v[j-1], v[j], v[j+1]) across lanes.  ASM: two v_max_f32 with a DPP
// source (the moves fold into the max); s_nop 1 covers the two wait states a
// DPP read needs after a VALU write of its source.
template <bool ASM>
__device__ __forceinline__ float hmax3(float v)
{
    if constexpr (ASM) {
        float m;
        asm volatile(
            "s_nop 1\n\t"
            "v_max_f32_dpp %0, %1, %1 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
            "v_max_f32_dpp %0, %1, %0 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
            : "=&v"(m)
            : "v"(v));
        return m;
    } else {
        return fmaxf(fmaxf(v, dpp_from_lower(v)), dpp_from_upper(v));
    }
}

// Eight window maxima at once (the strip's rows): two v_max_f32 with a DPP
// source per row, one s_nop 1 ahead of them for the two wait states a DPP
// read needs after a VALU write of its source.
__device__ __forceinline__ void hmax3x8(const float (&v)[8], float (&m)[8])
{
    asm("s_nop 1\n\t"
        "v_max_f32_dpp %0, %8, %8 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %1, %9, %9 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %2, %10, %10 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %3, %11, %11 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %4, %12, %12 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %5, %13, %13 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %6, %14, %14 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %7, %15, %15 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %0, %8, %0 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %1, %9, %1 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %2, %10, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %3, %11, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %4, %12, %4 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %5, %13, %5 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %6, %14, %6 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_max_f32_dpp %7, %15, %7 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=&v"(m[0]), "=&v"(m[1]), "=&v"(m[2]), "=&v"(m[3]), "=&v"(m[4]), "=&v"(m[5]), "=&v"(m[6]), "=&v"(m[7])
        : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]));
}

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

// The rotated table as seen by the search kernel: read through the constant
// address space, so that the wave-uniform entries arrive by scalar loads.
typedef const __attribute__((address_space(4))) TabEntry CTabEntry;

__device__ __forceinline__ TabEntry tab_entry(CTabEntry* t)
{
    TabEntry e;
    e.qx = t->qx;
    e.qy = t->qy;
    e.rx = t->rx;
    e.ry = t->ry;
    e.rh = t->rh;
    return e;
}

// Storage of one field pixel in the LDS tile and its dot product with a
// table entry's rotated direction: FP32 pairs, or FP16 pairs with the
// v_dot2_f32_f16 product accumulated in FP32.
template <int PREC>
struct Px;
template <>
struct Px<TM_FP32> {
    using T = float2;
    static __device__ __forceinline__ T zero() { return make_float2(0.f, 0.f); }
    static __device__ __forceinline__ T load(const void* f, size_t o) { return reinterpret_cast<const float2*>(f)[o]; }
    // one product and one fused multiply-add, written out so that every kernel
    // that scores in FP32 (the searches and the re-scoring of an FP16 search)
    // rounds it identically
    static __device__ __forceinline__ float dot(const TabEntry& e, T g) { return __builtin_fmaf(e.ry, g.y, e.rx * g.x); }
    // on the edge set: the field and the tile padding hold non-edges as (+0, +0)
    static __device__ __forceinline__ bool edge(T g) { return (__float_as_uint(g.x) | __float_as_uint(g.y)) != 0u; }
    template <bool ASM>
    static __device__ __forceinline__ float dot_t(const TabEntry& e, T g)
    {
        return dot(e, g);
    }
};
template <>
struct Px<TM_FP16> {
    using T = uint32_t;
    static __device__ __forceinline__ T zero() { return 0u; }
    static __device__ __forceinline__ T load(const void* f, size_t o) { return reinterpret_cast<const uint32_t*>(f)[o]; }
    static __device__ __forceinline__ float dot(const TabEntry& e, T g)
    {
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, e.rh), __builtin_bit_cast(h2_t, g), 0.0f, false);
    }
    // non-edges are the half2 (+0, +0), bit pattern 0
    static __device__ __forceinline__ bool edge(T g) { return g != 0u; }
    template <bool ASM>
    static __device__ __forceinline__ float dot_t(const TabEntry& e, T g)
    {
        return dot(e, g);
    }
};

// The ten products of one point down an 8-row strip (rows 0..9 of the
// window) in the VOP3P form with an inline zero addend (the builtin becomes
// v_dot2c with an accumulator cleared by a move per product).  A dot result
// must not be read by another VALU instruction within 3 wait states, which
// the compiler cannot see inside asm: five ordered pairs of products (each
// waiting only for its own two LDS values), then s_nop 2, then a scheduling
// barrier that no VALU instruction crosses, so every reader comes after the
// wait states (LDS reads and scalar instructions may still move across).
__device__ __forceinline__ void dots10_f16(uint32_t rh, const uint32_t (&g)[10], float (&d)[10])
{
#pragma unroll
    for (int j = 0; j < 10; j += 2)
        asm volatile(
            "v_dot2_f32_f16 %0, %2, %3, 0\n\t"
            "v_dot2_f32_f16 %1, %2, %4, 0"
            : "=&v"(d[j]), "=&v"(d[j + 1])
            : "s"(rh), "v"(g[j]), "v"(g[j + 1]));
    asm volatile("s_nop 2");
    __builtin_amdgcn_sched_barrier(0x0104);
}

// The same ten products with a per-pixel addend: the tile of the FP16
// edge-taps form holds, beside each half2, the FP32 value it adds to its
// products (0 on the edge set, kOffEdge elsewhere), so that a product comes
// out of v_dot2_f32_f16 as a window operand of that form in one instruction.
// Hazard handling as in dots10_f16.
__device__ __forceinline__ void dots10_f16_biased(uint32_t rh, const uint2 (&g)[10], float (&d)[10])
{
#pragma unroll
    for (int j = 0; j < 10; j += 2)
        asm volatile(
            "v_dot2_f32_f16 %0, %2, %3, %4\n\t"
            "v_dot2_f32_f16 %1, %2, %5, %6"
            : "=&v"(d[j]), "=&v"(d[j + 1])
            : "s"(rh), "v"(g[j].x), "v"(g[j].y), "v"(g[j + 1].x), "v"(g[j + 1].y));
    asm volatile("s_nop 2");
    __builtin_amdgcn_sched_barrier(0x0104);
}

// Tile element of the search kernel: the field pixel as stored, or for the
// FP16 edge-taps form (BIASED) the half2 and the FP32 bits of its addend.
template <int PREC, int VOTE>
struct TileOf {
    static constexpr bool BIASED = PREC == TM_FP16 && VOTE == 1;
    using T = std::conditional_t<BIASED, uint2, typename Px<PREC>::T>;
    static __device__ __forceinline__ T make(typename Px<PREC>::T v)
    {
        if constexpr (BIASED)
            return make_uint2(v, v != 0u ? 0u : __float_as_uint(kOffEdge));
        else
            return v;
    }
};

struct FastArgs {
    int level;          // searched level
    int tr;             // 1: lanes run along y and strips along x (the tile transposed)
    int K;              // angles
    int A;              // angles per workgroup
    int WY, WA;         // waves stacked in y, waves splitting the angles
    int C;              // chunks of angles
    const int2* work;   // optional work list: block b runs (pair, block) work[b]; pair < 0: nothing
};

// What a certified FP16 search keeps per translation and angle range: the
// best angle by the key (S_w desc, S_1 desc, k asc; the fast kernel's screen
// has no S_1 and keeps 0), the runner-up by S_w (its angle), and the best S_w
// of all the remaining angles.  Invariant: w3 <= w2 <= w.
struct Top3 {
    float w, s;
    int k;
    float w2;
    int k2;
    float w3;
};

// Add one angle's (S_w, S_1, k) to a summary.
__device__ __forceinline__ void top3_add(Top3& t, float w, float s, int k)
{
    if (key_better(w, s, 0, 0, k, t.w, t.s, 0, 0, t.k)) {
        t.w3 = fmaxf(t.w3, t.w2);
        t.w2 = t.w;
        t.k2 = t.k;
        t.w = w;
        t.s = s;
        t.k = k;
    } else if (w > t.w2) {
        t.w3 = fmaxf(t.w3, t.w2);
        t.w2 = w;
        t.k2 = k;
    } else {
        t.w3 = fmaxf(t.w3, w);
    }
}

// Merge the summary of another set of angles into a.
__device__ __forceinline__ void top3_merge(Top3& a, const Top3& b)
{
    if (key_better(b.w, b.s, 0, 0, b.k, a.w, a.s, 0, 0, a.k)) {
        Top3 r = b;
        if (a.w > b.w2) {  // a's best is the runner-up
            r.w2 = a.w;
            r.k2 = a.k;
            r.w3 = fmaxf(b.w2, a.w2);
        } else {
            r.w3 = fmaxf(b.w3, a.w);
        }
        a = r;
    } else if (b.w > a.w2) {  // b's best is the runner-up
        a.w3 = fmaxf(a.w2, b.w2);
        a.w2 = b.w;
        a.k2 = b.k;
    } else {
        a.w3 = fmaxf(a.w3, b.w);
    }
}

// Chunk partials of a certified search: best (S_w, S_1, k), runner-up (S_w,
// k), rest's best S_w.
__device__ __forceinline__ void top3_store(const PairDesc& P, size_t o, const Top3& t)
{
    P.pw[o] = t.w;
    P.p1[o] = t.s;
    P.pk[o] = t.k;
    P.p2[o] = t.w2;
    P.pk2[o] = t.k2;
    P.p3[o] = t.w3;
}

__device__ __forceinline__ Top3 top3_load(const PairDesc& P, size_t o)
{
    return Top3{P.pw[o], P.p1[o], P.pk[o], P.p2[o], P.pk2[o], P.p3[o]};
}

// VAR: 0 compiler-built products and window maxima; 1 the same with the
// VOP3P dot and the DPP-folded maxima written out; 2, 3, 4 as 1 with 2, 4, 8
// table entries fetched per loop step (one scalar-load wait per step); 5 as 3
// with the next step's entries requested behind this step's LDS reads.
// VOTE 1: the edge-taps-only window (off-edge products replaced by kOffEdge
// before the maxima, each window maximum finished by vote_finish); the centre
// sum takes the plain products in both readings.  In FP16 the replacement is
// the addend stored with each tile pixel (TileOf), and the centre sum takes
// vote_finish of the product, which is the plain product on the edge set and
// -0 elsewhere.
// SCREEN (an FP16 search whose decisions are certified): no centre sum; per
// row the best angle by (S_w desc, k asc), the runner-up's S_w and angle, and
// the best S_w of the remaining angles (Top3 below), which is what the
// certification needs to know which angles could win in FP32.
template <int G, int R, int LC, int PREC, int VAR, int VOTE, bool SCREEN = false>
__global__ __launch_bounds__(1024) void k_dense_fast(FastArgs a, const PairDesc* __restrict__ pairs)
{
    using Tile = TileOf<PREC, VOTE>;
    using T = typename Tile::T;
    using PT = typename Px<PREC>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    T* tile = reinterpret_cast<T*>(smem);
    constexpr int NS = 64 / G;   // segments per wave
    constexpr int TW = G - 2;    // output columns per segment
    int pr = blockIdx.y, bx = blockIdx.x;
    if (a.work) {
        const int2 wv = a.work[blockIdx.x];
        pr = wv.x;
        bx = wv.y;
        if (pr < 0) return;
    }
    // Tile frame: u runs along the lanes (the tile's columns, TW per
    // segment), v along the strips (its rows, TH).  tr 0: u = x, v = y; tr 1:
    // u = y, v = x, which fits some level shapes with fewer idle lanes (the
    // 3x3 window is symmetric, so the scores are the same).
    const PairDesc& P = pairs[pr];
    const int n_tiles = P.tiles_x * P.tiles_y;  // tiles along u, v
    if (bx >= n_tiles * a.C) return;
    const int TH = a.WY * NS * R;
    const int chunk = bx / n_tiles;
    const int tid = bx % n_tiles;
    const int U0 = (tid % P.tiles_x) * TW, V0 = (tid / P.tiles_x) * TH;
    const int W = P.W[a.level], H = P.H[a.level];
    const void* field = P.sfield;
    const int halo = P.rad + 1;
    const int LR = TH + 2 * halo;
    const int fc = TW + 2 * halo;
    const bool tr = a.tr != 0;

    // stage tile[v][u]; consecutive threads take consecutive x
    for (int e = threadIdx.x; e < LR * fc; e += blockDim.x) {
        int r, c;
        if (tr) {
            c = e / LR;
            r = e - c * LR;
        } else {
            r = e / fc;
            c = e - r * fc;
        }
        const int u = U0 - halo + c, v = V0 - halo + r;
        const int x = tr ? v : u, y = tr ? u : v;
        PT val = Px<PREC>::zero();
        if (x >= 0 && x < W && y >= 0 && y < H) val = Px<PREC>::load(field, (size_t)y * W + x);
        tile[r * LC + c] = Tile::make(val);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int wy = wid % a.WY, wa = wid / a.WY;
    const int seg = lane / G, li = lane - seg * G;
    const int row0 = (wy * NS + seg) * R;  // first output row of the strip, tile-relative
    const T* lbase = tile + (halo - 1 + row0) * LC + (halo - 1 + li);
    CTabEntry* tab = (CTabEntry*)P.tab;
    const int n_pad = P.n_pad;
    const float n_f = (float)P.n[a.level];

    static_assert(!SCREEN || PREC == TM_FP16, "only the FP16 search is certified");
    float bw[R], b1[R], w2[R], w3[R];
    int bk[R], k2[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        bw[r] = -INFINITY;
        b1[r] = -INFINITY;
        w2[r] = -INFINITY;
        w3[r] = -INFINITY;
        bk[r] = -1;
        k2[r] = -1;
    }
    const int k0 = chunk * a.A, k1 = min(a.K, k0 + a.A);
    for (int k = k0 + wa; k < k1; k += a.WA) {
        CTabEntry* Tb = tab + (size_t)k * n_pad;
        float tw[R], t1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            tw[r] = 0.f;
            t1[r] = 0.f;
        }
        for (int i0 = 0; i0 < n_pad; i0 += kBlock) {
            float pw[R], p1[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                pw[r] = 0.f;
                p1[r] = 0.f;
            }
            const int i1 = min(n_pad, i0 + kBlock);
            constexpr bool ASM = VAR > 0;
            // one point: its R+2 products down the strip, the vertical then
            // the horizontal window maxima, added in point order
            // (fetch: the point's R+2 field values from LDS; compute: the rest)
            auto fetch = [&](const TabEntry& e, T (&gv)[R + 2]) {
                const int qu = tr ? (int)e.qy : (int)e.qx, qv = tr ? (int)e.qx : (int)e.qy;
                const T* p = lbase + qv * LC + qu;
#pragma unroll
                for (int rr = 0; rr < R + 2; ++rr) gv[rr] = p[rr * LC];
            };
            auto compute = [&](const TabEntry& e, const T (&gv)[R + 2]) {
                float D[R + 2];
                float E[R + 2];
                if constexpr (Tile::BIASED) {
                    static_assert(ASM && R == 8, "the biased tile has the written-out form only");
                    dots10_f16_biased(e.rh, gv, E);
#pragma unroll
                    for (int rr = 1; rr <= R; ++rr) D[rr] = vote_finish(E[rr]);
                } else {
                    if constexpr (ASM && PREC == TM_FP16 && R == 8) {
                        dots10_f16(e.rh, gv, D);
                    } else {
#pragma unroll
                        for (int rr = 0; rr < R + 2; ++rr) D[rr] = Px<PREC>::template dot_t<ASM>(e, gv[rr]);
                    }
#pragma unroll
                    for (int rr = 0; rr < R + 2; ++rr) {
                        if constexpr (VOTE == 1)
                            E[rr] = Px<PREC>::edge(gv[rr]) ? D[rr] : kOffEdge;
                        else
                            E[rr] = D[rr];
                    }
                }
                float V[R];
#pragma unroll
                for (int r = 0; r < R; ++r) V[r] = fmaxf(fmaxf(E[r], E[r + 1]), E[r + 2]);
                if constexpr (ASM && R == 8) {
                    float M[R];
                    hmax3x8(V, M);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        pw[r] += win_finish<VOTE>(M[r]);
                        if constexpr (!SCREEN) p1[r] += D[r + 1];
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        pw[r] += win_finish<VOTE>(hmax3<ASM>(V[r]));
                        if constexpr (!SCREEN) p1[r] += D[r + 1];
                    }
                }
            };
            auto point = [&](const TabEntry& e) {
                T gv[R + 2];
                fetch(e, gv);
                compute(e, gv);
            };
            if constexpr (VAR == 5) {
                // 4 points per step, software-pipelined: the next step's table
                // entries are requested after this step's LDS reads, so that
                // the two waits overlap
                constexpr int U = 4;
                TabEntry e[U];
#pragma unroll
                for (int u = 0; u < U; ++u) e[u] = tab_entry(Tb + i0 + u);
                for (int i = i0; i < i1; i += U) {
                    T gv[U][R + 2];
#pragma unroll
                    for (int u = 0; u < U; ++u) fetch(e[u], gv[u]);
                    __builtin_amdgcn_sched_barrier(0);
                    const int inext = i + U < i1 ? i + U : i;  // the last step re-reads its own entries
                    TabEntry en[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) en[u] = tab_entry(Tb + inext + u);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < U; ++u) compute(e[u], gv[u]);
#pragma unroll
                    for (int u = 0; u < U; ++u) e[u] = en[u];
                }
            } else if constexpr (VAR >= 2) {
                // U entries fetched together, then U points in order; block
                // lengths are multiples of 8 (the table is padded to 8)
                constexpr int U = VAR == 2 ? 2 : (VAR == 3 ? 4 : 8);
                for (int i = i0; i < i1; i += U) {
                    TabEntry e[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) e[u] = tab_entry(Tb + i + u);
#pragma unroll
                    for (int u = 0; u < U; ++u) point(e[u]);
                }
            } else {
#pragma unroll 2
                for (int i = i0; i < i1; ++i) point(tab_entry(Tb + i));
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                tw[r] += pw[r];
                if constexpr (!SCREEN) t1[r] += p1[r];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float sw = tw[r] / n_f;
            if constexpr (SCREEN) {
                // angles arrive in increasing order: a strictly larger S_w wins
                if (sw > bw[r]) {
                    w3[r] = fmaxf(w3[r], w2[r]);
                    w2[r] = bw[r];
                    k2[r] = bk[r];
                    bw[r] = sw;
                    bk[r] = k;
                } else if (sw > w2[r]) {
                    w3[r] = fmaxf(w3[r], w2[r]);
                    w2[r] = sw;
                    k2[r] = k;
                } else {
                    w3[r] = fmaxf(w3[r], sw);
                }
            } else {
                const float s1 = t1[r] / n_f;
                if (sw > bw[r] || (sw == bw[r] && s1 > b1[r])) {
                    bw[r] = sw;
                    b1[r] = s1;
                    bk[r] = k;
                }
            }
        }
    }

    // combine the WA waves that share this tile, in key order
    __syncthreads();
    const int npos = TH * TW;
    const int nq = a.WA * npos;
    float* cw = reinterpret_cast<float*>(smem);
    float* c1 = cw + nq;  // S_1; in SCREEN the runner-up's S_w
    int* ck = reinterpret_cast<int*>(c1 + nq);
    int* ck2 = ck + nq;   // SCREEN: the runner-up's angle
    float* c3 = reinterpret_cast<float*>(ck2 + nq);  // SCREEN: the best S_w of the rest
    if (li >= 1 && li <= G - 2) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int idx = (wa * TH + row0 + r) * TW + (li - 1);
            cw[idx] = bw[r];
            ck[idx] = bk[r];
            if constexpr (SCREEN) {
                c1[idx] = w2[r];
                ck2[idx] = k2[r];
                c3[idx] = w3[r];
            } else {
                c1[idx] = b1[r];
            }
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < npos; p += blockDim.x) {
        const int pv = p / TW, pu = p - pv * TW;
        const int X = tr ? V0 + pv : U0 + pu, Y = tr ? U0 + pu : V0 + pv;
        if (X >= W || Y >= H) continue;
        const size_t o = ((size_t)chunk * H + Y) * W + X;
        if constexpr (SCREEN) {
            Top3 t{cw[p], 0.f, ck[p], c1[p], ck2[p], c3[p]};
            for (int w = 1; w < a.WA; ++w) {
                const int q = w * npos + p;
                top3_merge(t, Top3{cw[q], 0.f, ck[q], c1[q], ck2[q], c3[q]});
            }
            top3_store(P, o, t);
        } else {
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
            P.pw[o] = w0;
            P.p1[o] = s0;
            P.pk[o] = kk;
        }
    }
}

struct GenericArgs {
    int level, K, A, sx, sy, win;
};

// The searched level's field copied with a zero border of P.pad pixels on
// every side (P.pW x P.pH elements), so that the generic search reads any tap
// of any window without clamping: zero is a non-edge direction, which votes
// 0, exactly as a tap outside the image does.  grid: (padded pixels, pair).
template <int PREC>
__global__ __launch_bounds__(256) void k_pad_field(int level, const PairDesc* __restrict__ pairs)
{
    using T = typename Px<PREC>::T;
    const PairDesc& P = pairs[blockIdx.y];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P.pW * P.pH) return;
    const int yy = idx / P.pW, xx = idx - yy * P.pW;
    const int x = xx - P.pad, y = yy - P.pad, W = P.W[level], H = P.H[level];
    T v = Px<PREC>::zero();
    if (x >= 0 && x < W && y >= 0 && y < H) v = Px<PREC>::load(P.sfield, (size_t)y * W + x);
    reinterpret_cast<T*>(P.pfield)[idx] = v;
}

// Any step and window: one thread per grid translation, taps read from the
// zero-bordered copy of the field (no clamping, one address add per tap);
// products as in the fast kernel (Px::dot).  The 3x3 window takes four points
// per step over the padded table (padding entries, q = 0 and r = 0, add
// exactly 0; blocks keep their bounds since 8 divides 32).  VOTE as in
// k_dense_fast.  grid: (translations, chunk, pair).
// SCREEN: also the runner-up and the rest's best (Top3) for the certification.
template <int PREC, int VOTE, bool SCREEN = false>
__global__ __launch_bounds__(256) void k_dense_generic(GenericArgs a, const PairDesc* __restrict__ pairs)
{
    using T = typename Px<PREC>::T;
    const PairDesc& P = pairs[blockIdx.z];
    const int gw = P.gw, gh = P.gh;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = blockIdx.y;
    if (p >= gw * gh) return;
    const T* __restrict__ pf = reinterpret_cast<const T*>(P.pfield);
    const int pW = P.pW, pad = P.pad;
    const int n = P.n[a.level];
    const float n_f = (float)n;
    const int gy = p / gw, gx = p - gy * gw;
    const int x = gx * a.sx, y = gy * a.sy;
    const int h = (a.win - 1) / 2;
    // the window's top-left tap of a point at offset (0, 0)
    const int origin = (y + pad - h) * pW + (x + pad - h);
    auto win_op = [&](const TabEntry& e, T g) {
        const float d = Px<PREC>::dot(e, g);
        if constexpr (VOTE == 1)
            return Px<PREC>::edge(g) ? d : kOffEdge;
        else
            return d;
    };
    Top3 t{-INFINITY, -INFINITY, -1, -INFINITY, -1, -INFINITY};
    const int k0 = chunk * a.A, k1 = min(a.K, k0 + a.A);
    for (int k = k0; k < k1; ++k) {
        CTabEntry* Tb = (CTabEntry*)P.tab + (size_t)k * P.n_pad;  // wave-uniform: scalar loads
        float tw = 0.f, t1 = 0.f;
        const int nl = h == 1 ? P.n_pad : n;
        for (int i0 = 0; i0 < nl; i0 += kBlock) {
            float pw = 0.f, p1 = 0.f;
            const int i1 = min(nl, i0 + kBlock);
            if (h == 1) {
                constexpr int U = 4;
                for (int i = i0; i < i1; i += U) {
                    TabEntry e[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) e[u] = tab_entry(Tb + i + u);
                    T g[U][3][3];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const T* b = pf + origin + (int)e[u].qy * pW + (int)e[u].qx;
#pragma unroll
                        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                            for (int dx = 0; dx < 3; ++dx) g[u][dy][dx] = b[dy * pW + dx];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        float best = -INFINITY;
#pragma unroll
                        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                            for (int dx = 0; dx < 3; ++dx) best = fmaxf(best, win_op(e[u], g[u][dy][dx]));
                        pw += win_finish<VOTE>(best);
                        p1 += Px<PREC>::dot(e[u], g[u][1][1]);
                    }
                }
            } else {
                for (int i = i0; i < i1; ++i) {
                    const TabEntry e = tab_entry(Tb + i);
                    const T* b = pf + origin + (int)e.qy * pW + (int)e.qx;
                    float best = -INFINITY;
                    for (int dy = 0; dy <= 2 * h; ++dy)
#pragma unroll 3
                        for (int dx = 0; dx <= 2 * h; ++dx) best = fmaxf(best, win_op(e, b[dy * pW + dx]));
                    pw += win_finish<VOTE>(best);
                    p1 += Px<PREC>::dot(e, b[h * pW + h]);
                }
            }
            tw += pw;
            t1 += p1;
        }
        const float sw = tw / n_f, s1 = t1 / n_f;
        if constexpr (SCREEN) {
            top3_add(t, sw, s1, k);
        } else if (sw > t.w || (sw == t.w && s1 > t.s)) {
            t.w = sw;
            t.s = s1;
            t.k = k;
        }
    }
    const size_t o = ((size_t)chunk * gh + gy) * gw + gx;
    if constexpr (SCREEN) {
        top3_store(P, o, t);
    } else {
        P.pw[o] = t.w;
        P.p1[o] = t.s;
        P.pk[o] = t.k;
    }
}

// Best angle per translation over the C chunk partials, in key order.  A
// workgroup takes 32 translations; 8 threads share one translation, each
// scanning every 8th chunk with its loads issued ahead of the comparisons,
// then the 8 partial bests are merged through LDS.  The key is a total order,
// so the result does not depend on the split.
constexpr int kRedLanes = 8;
constexpr int kRedPos = 32;

__global__ __launch_bounds__(256) void k_reduce_chunks(int C, const PairDesc* __restrict__ pairs)
{
    __shared__ float sw_[kRedPos][kRedLanes], s1_[kRedPos][kRedLanes];
    __shared__ int sk_[kRedPos][kRedLanes];
    const PairDesc& P = pairs[blockIdx.y];
    const int np = P.gw * P.gh;
    if ((int)blockIdx.x * kRedPos >= np) return;
    const float* __restrict__ pw = P.pw;
    const float* __restrict__ p1 = P.p1;
    const int32_t* __restrict__ pk = P.pk;
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
        P.mw[p] = w0;
        P.m1[p] = s0;
        P.mk[p] = k;
    }
}

// Per translation of a certified search: the chunks' Top3 summaries merged
// (the key is a total order, so the merge order does not matter), written to
// the map with the runner-up and the rest's best.  clear (optional): the
// certification's list counter, set to 0 here for the launches that follow.
__global__ __launch_bounds__(256) void k_reduce_screen(int C, const PairDesc* __restrict__ pairs, int* clear)
{
    if (clear && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *clear = 0;
    const PairDesc& P = pairs[blockIdx.y];
    const int np = P.gw * P.gh;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    Top3 t = top3_load(P, p);
    for (int c = 1; c < C; ++c) top3_merge(t, top3_load(P, (size_t)c * np + p));
    P.mw[p] = t.w;
    P.m1[p] = t.s;
    P.mk[p] = t.k;
    P.m2[p] = t.w2;
    P.mk2[p] = t.k2;
    P.m3[p] = t.w3;
}

// One wave per pose: lanes take points i = lane, lane + 64, ...; each point's
// rotation is formed in FP64, its window read from global memory; per-lane
// sums are combined by a fixed butterfly.  VOTE as in k_dense_fast.
template <int PREC, int VOTE>
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
                best = fmaxf(best, field_win_tap<PREC, VOTE>(field, W, H, px + dx, py + dy, fx, fy));
        sw += win_finish<VOTE>(best);
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

// ---------------------------------------------------------------- certification of an FP16 search
//
// An FP16 search scores every pose with half2 directions and FP32 sums.  Its
// score of a pose differs from the FP32 search's (the same sums over the FP32
// directions) by at most E(n), n the level's model points (cert_eps below).
// The selection decides on the map: the best angle per translation, which
// translations are strict local maxima above the floor, their key order.
// These decisions are made identical to the ones taken on the FP32 map, with
// M the FP16 map value and hi = M + E, lo = M - E bounding the FP32 one:
//  * u may be a candidate in FP32 iff hi(u) >= min_score and no grid
//    neighbour v has lo(v) > hi(u) (such a v beats u in FP32 as well);
//  * every such u, and every neighbour v of one with hi(v) >= lo(u), is given
//    its FP32 value: the FP32 search's own arithmetic (Px<TM_FP32>::dot,
//    blocks of 32 points, the same divisions and key) over the angles that
//    can hold the FP32 best, i.e. the angle chunks whose FP16 best reaches
//    M - 2E; when that is a single chunk whose other angles all stay below
//    M - 2E (its second best), the FP16 best angle alone is scored;
//  * every other translation keeps its FP16 value: it is below the floor in
//    both maps, or strictly beaten by a neighbour in both, and next to a
//    possible candidate it is strictly below that candidate in both.
// The selection on the patched map therefore returns the FP32 search's
// candidates with their FP32 values, and a detection continues exactly as an
// FP32 one does (the refinement reads the FP32 twin).
//
// E(n): per product, the FP16 rounding of both unit vectors (2^-11 relative
// per component) moves r . g by at most 2^-11 (|r||g_h| + |r||g|) <= 2^-10 +
// 2^-22, and the two FP32 roundings of each product add 2^-23; a window
// maximum moves by no more than its operands; each blocked FP32 sum of n
// votes of size <= 1 + 2^-10 is within (31 + ceil(n/32)) 2^-24 per vote of
// the exact sum, twice (both searches), plus the two divisions.  A unit
// field direction from integer gradients has no component below 1/1443, so
// none is an FP16 subnormal; a rotated model direction may have one (below
// 2^-14), and were the product to flush it, the product would move by at most
// 2^-14 more.  cert_eps takes 2^-10 + 2^-14 + 2^-18 + (66 + 2 ceil(n/32))
// 2^-23, above all of it.
__device__ __forceinline__ double cert_eps(int n)
{
    return ldexp(1.0, -10) + ldexp(1.0, -14) + ldexp(1.0, -18) +
           (66.0 + 2.0 * (double)((n + 31) / 32)) * ldexp(1.0, -23);
}

struct CertArgs {
    int level, C, A, K, win, sx, sy;
    float min_score;
    CertBufs cb;
    int lds_bytes;  // k_rescore: bytes of its staged field block (0: gathers only)
};

__global__ __launch_bounds__(64) void k_cert_zero(int* count)
{
    if (threadIdx.x == 0) count[0] = 0;
}

// Whether translation p of pair pr must be re-scored in FP32, and its entry.
__device__ __forceinline__ bool certify_entry(const CertArgs& a, const PairDesc& P, int pr, int p, int gw, int gh,
                                              int np, int4* out)
{
    const int x = p % gw, y = p / gw;
    const double E = cert_eps(P.n[a.level]);
    double M[5][5];
    bool in[5][5];
#pragma unroll
    for (int b = 0; b < 5; ++b)
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const int xx = x + c - 2, yy = y + b - 2;
            in[b][c] = (unsigned)xx < (unsigned)gw && (unsigned)yy < (unsigned)gh;
            M[b][c] = in[b][c] ? (double)P.mw[yy * gw + xx] : 0.0;
        }
    // may the translation at block position (b, c) (1..3) be a candidate in FP32?
    auto possible = [&](int b, int c) -> bool {
        if (!in[b][c]) return false;
        const double hi = M[b][c] + E;
        if (!(hi >= (double)a.min_score)) return false;
        bool ok = true;
#pragma unroll
        for (int v = -1; v <= 1; ++v)
#pragma unroll
            for (int u = -1; u <= 1; ++u)
                if ((u || v) && in[b + v][c + u] && M[b + v][c + u] - E > hi) ok = false;
        return ok;
    };
    bool need = possible(2, 2);
    const double hi_u = M[2][2] + E;
#pragma unroll
    for (int v = -1; v <= 1; ++v)
#pragma unroll
        for (int u = -1; u <= 1; ++u)
            if ((u || v) && !need && possible(2 + v, 2 + u) && hi_u >= M[2 + v][2 + u] - E) need = true;
    if (!need) return false;
    const double lim = M[2][2] - 2.0 * E;
    int4& en = *out;
    if ((double)P.m3[p] < lim) {
        // the FP32 best is the FP16 best angle, or the runner-up if it reaches M - 2E
        en = make_int4(pr, p, P.mk[p], (double)P.m2[p] >= lim ? P.mk2[p] : -1);
    } else {
        unsigned long long mask = 0ull;
        for (int c = 0; c < a.C && c < 64; ++c)
            if ((double)P.pw[(size_t)c * np + p] >= lim) mask |= 1ull << c;
        if (a.C > 64) mask = ~0ull;  // all angles
        en = make_int4(-1 - pr, p, (int)(unsigned)(mask & 0xffffffffull), (int)(unsigned)(mask >> 32));
    }
    return true;
}

// One thread per translation of every pair: the translations whose FP32
// values the selection needs, queued with the angles to score.  Entry
// (pair, translation, a, b): the angles a and b (b < 0: none) when every
// other angle is below M - 2E (the map's runner-up and rest's best say so);
// otherwise (-1 - pair, translation, mask low, mask high): the angle chunks
// whose FP16 best reaches M - 2E.  A workgroup's entries take their places
// in the list with one atomic (its count, in LDS first), not one each.
__global__ __launch_bounds__(256) void k_certify(CertArgs a, const PairDesc* __restrict__ pairs)
{
    __shared__ int wg_count, wg_base;
    if (threadIdx.x == 0) wg_count = 0;
    __syncthreads();
    const int pr = blockIdx.y;
    const PairDesc& P = pairs[pr];
    const int gw = P.gw, gh = P.gh, np = gw * gh;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    int4 en = make_int4(0, 0, 0, 0);
    const bool listed = p < np && certify_entry(a, P, pr, p, gw, gh, np, &en);
    const int slot = listed ? atomicAdd(&wg_count, 1) : 0;
    __syncthreads();
    if (threadIdx.x == 0 && wg_count > 0) wg_base = atomicAdd(&a.cb.count[0], wg_count);
    __syncthreads();
    if (listed) a.cb.list[wg_base + slot] = en;
}

// One model point's windowed vote (the maximum of its window's products,
// finished for the edge-taps reading) and its centre product, in FP32 with
// the FP32 search's arithmetic.  g(qx, qy): the FP32 field at the
// translation plus (qx, qy), zero outside the image.  HW: the window's half
// side when it is 1 (the loops unrolled), else -1 (h at run time).
template <int VOTE, int HW, class Fetch>
__device__ __forceinline__ void vote_fp32(const TabEntry& e, int h, Fetch g, float* vote, float* centre)
{
    float best = -INFINITY, c = 0.f;
    auto tap = [&](int dx, int dy) {
        const float2 v = g((int)e.qx + dx, (int)e.qy + dy);
        const float d = Px<TM_FP32>::dot(e, v);
        if (dx == 0 && dy == 0) c = d;
        if constexpr (VOTE == 1)
            best = fmaxf(best, Px<TM_FP32>::edge(v) ? d : kOffEdge);
        else
            best = fmaxf(best, d);
    };
    if constexpr (HW == 1) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) tap(dx, dy);
    } else {
        for (int dy = -h; dy <= h; ++dy)
            for (int dx = -h; dx <= h; ++dx) tap(dx, dy);
    }
    *vote = win_finish<VOTE>(best);
    *centre = c;
}

constexpr int kWaveSeg = 512;  // points whose votes score_fp32_wave keeps in LDS at a time

// One pose scored by a whole wave, lane t taking points t, t + 64, ...: the
// votes of kWaveSeg points at a time go to the wave's LDS buffers vb, cb
// (kWaveSeg floats each), lane b then adds block b of 32 of them in point
// order, and the block sums are added in order, so the sums are those of
// score_fp32 bit for bit.  Every lane returns the result.
template <int VOTE, int HW, class Fetch>
__device__ __forceinline__ void score_fp32_wave(const TabEntry* __restrict__ Tb, int n_pad, float n_f, int h, Fetch g,
                                                float* vb, float* cb, float* sw, float* s1)
{
    const int lane = threadIdx.x & 63;
    float tw = 0.f, t1 = 0.f;
    for (int s0 = 0; s0 < n_pad; s0 += kWaveSeg) {
        const int sn = min(kWaveSeg, n_pad - s0);
        for (int i = lane; i < sn; i += 64) {
            float v, c;
            vote_fp32<VOTE, HW>(Tb[s0 + i], h, g, &v, &c);
            vb[i] = v;
            cb[i] = c;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the votes written before any lane reads them
        const int nbk = (sn + kBlock - 1) / kBlock;
        float pw = 0.f, p1 = 0.f;
        if (lane < nbk) {
            const int i1 = min(sn, (lane + 1) * kBlock);
            for (int i = lane * kBlock; i < i1; ++i) {
                pw += vb[i];
                p1 += cb[i];
            }
        }
        for (int b = 0; b < nbk; ++b) {
            tw += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pw), b));
            t1 += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p1), b));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // read before the next segment overwrites
    }
    *sw = tw / n_f;
    *s1 = t1 / n_f;
}

// Eq. (1) of one pose in FP32 with the FP32 search's arithmetic: window
// maximum of the products of each (padded) table entry, votes added in
// blocks of 32 points in point order, block sums in order, one division.
// g(qx, qy): the FP32 field at the translation plus (qx, qy), zero outside
// the image.  HW: the window's half side when it is 1 (the loops unrolled),
// else -1 (h at run time).
template <int VOTE, int HW, class Fetch>
__device__ __forceinline__ void score_fp32(const TabEntry* __restrict__ Tb, int n_pad, float n_f, int h_rt, Fetch g,
                                           float* sw, float* s1)
{
    const int h = HW >= 0 ? HW : h_rt;
    float tw = 0.f, t1 = 0.f;
    for (int i0 = 0; i0 < n_pad; i0 += kBlock) {
        float pw = 0.f, p1 = 0.f;
        const int i1 = min(n_pad, i0 + kBlock);
        for (int i = i0; i < i1; ++i) {
            float v, c;
            vote_fp32<VOTE, HW>(Tb[i], h, g, &v, &c);
            pw += v;
            p1 += c;
        }
        tw += pw;
        t1 += p1;
    }
    *sw = tw / n_f;
    *s1 = t1 / n_f;
}

constexpr int kRescoreSums = 2048;  // (angle, block) sums k_rescore keeps in LDS at a time
static_assert(kRescoreSums >= 4 * kWaveSeg, "each of the four waves' vote buffers lies in the sums' space");

// The queued translations, the best by the key (S_w desc, S_1 desc, angle
// asc) written to the map: an entry naming one or two angles is scored by one
// wave (its lanes taking the points, the angles in turn, taps read from
// memory); an entry of open chunks by a whole workgroup, the FP32 field
// block around it staged in LDS when it fits, a thread per (angle, block of
// 32 points) forming that block's sum in point order, then a thread per
// angle adding its block sums in order (the sums of score_fp32, bit for
// bit).  Entry e goes to workgroup e mod the grid (an explicit one to its
// wave e / grid mod 4), so that no workgroup takes both kinds while others
// idle.
template <int VOTE, int HW>
__global__ __launch_bounds__(256) void k_rescore(CertArgs a, const PairDesc* __restrict__ pairs)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float2* blk = reinterpret_cast<float2*>(smem);
    __shared__ float rw[4], r1[4];
    __shared__ int rk[4];
    __shared__ int ch_lo[64], ch_n[64], n_ang;
    __shared__ float bs_w[kRescoreSums], bs_1[kRescoreSums];
    const int count = a.cb.count[0];
    const int h = (a.win - 1) / 2;
    // entries with one or two explicit angles: one wave each, the angles in
    // turn, the taps read from memory (the values a staged block gives:
    // zero outside the image); each wave's votes pass through its quarter of
    // bs_w / bs_1, which the open-chunk entries below reuse only after a
    // barrier every wave reaches once done here
    {
        const int nw = blockDim.x >> 6;
        for (int e = blockIdx.x + gridDim.x * (threadIdx.x >> 6); e < count; e += gridDim.x * nw) {
            const int4 en = a.cb.list[e];
            if (en.x < 0) continue;  // open chunks: below, by the whole workgroup
            const PairDesc& P = pairs[en.x];
            const int p = en.y;
            const int x = (p % P.gw) * a.sx, y = (p / P.gw) * a.sy;
            const int W = P.W[a.level], H = P.H[a.level];
            const float2* __restrict__ f32 = reinterpret_cast<const float2*>(P.field[a.level]);
            auto gathered_at = [&](int qx, int qy) {
                const int gx = x + qx, gy = y + qy;
                return ((unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H) ? f32[(size_t)gy * W + gx]
                                                                                  : make_float2(0.f, 0.f);
            };
            const float n_f = (float)P.n[a.level];
            float kw = -INFINITY, k1 = -INFINITY;
            int kk = 0x7fffffff;
            for (int t = 0; t < 2; ++t) {
                const int k = t == 0 ? en.z : en.w;
                if (k < 0) break;
                float sw, s1;
                score_fp32_wave<VOTE, HW>(P.tab + (size_t)k * P.n_pad, P.n_pad, n_f, h, gathered_at,
                                          bs_w + kWaveSeg * (threadIdx.x >> 6), bs_1 + kWaveSeg * (threadIdx.x >> 6),
                                          &sw, &s1);
                if (key_better(sw, s1, 0, 0, k, kw, k1, 0, 0, kk)) {
                    kw = sw;
                    k1 = s1;
                    kk = k;
                }
            }
            if ((threadIdx.x & 63) == 0) {
                P.mw[p] = kw;
                P.m1[p] = k1;
                P.mk[p] = kk;
            }
        }
    }
    for (int e = blockIdx.x; e < count; e += gridDim.x) {
        const int4 en = a.cb.list[e];
        const bool chunks = en.x < 0;
        if (!chunks) continue;  // taken above (the test is the same for the whole workgroup)
        const PairDesc& P = pairs[-1 - en.x];
        const int p = en.y;
        const int x = (p % P.gw) * a.sx, y = (p / P.gw) * a.sy;
        const int W = P.W[a.level], H = P.H[a.level];
        const float2* __restrict__ f32 = reinterpret_cast<const float2*>(P.field[a.level]);
        const int B = P.rad + h, S = 2 * B + 1;
        const bool staged = (long long)S * S * 8 <= a.lds_bytes;
        if (threadIdx.x == 0) {
            int m = 0, t = 0;
            if (a.C > 64) {  // every angle as one range
                ch_lo[0] = 0;
                ch_n[0] = a.K;
                t = a.K;
            } else {
                const unsigned long long mask =
                    (unsigned long long)(unsigned)en.z | ((unsigned long long)(unsigned)en.w << 32);
                for (int c = 0; c < a.C; ++c)
                    if ((mask >> c) & 1ull) {
                        ch_lo[m] = c * a.A;
                        ch_n[m] = min(a.K, (c + 1) * a.A) - c * a.A;
                        t += ch_n[m++];
                    }
            }
            n_ang = t;
        }
        if (staged)
            for (int i = threadIdx.x; i < S * S; i += blockDim.x) {
                const int r = i / S, c = i - r * S;
                const int gx = x - B + c, gy = y - B + r;
                blk[i] = ((unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H) ? f32[(size_t)gy * W + gx]
                                                                                      : make_float2(0.f, 0.f);
            }
        __syncthreads();
        float kw = -INFINITY, k1 = -INFINITY;
        int kk = 0x7fffffff;
        const float n_f = (float)P.n[a.level];
        const float2* ctr = blk + B * S + B;
        auto staged_at = [&](int qx, int qy) { return ctr[qy * S + qx]; };
        auto gathered_at = [&](int qx, int qy) {
            const int gx = x + qx, gy = y + qy;
            return ((unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H) ? f32[(size_t)gy * W + gx]
                                                                              : make_float2(0.f, 0.f);
        };
        {
            // open chunks, kRescoreSums / nb angles at a time: the block sums of
            // every (angle, block) pair, each a thread's, then each angle's total
            const int n_pad = P.n_pad, nb = (n_pad + kBlock - 1) / kBlock, per = kRescoreSums / nb;
            auto angle_of = [&](int j) {
                int c = 0, r = j;
                while (r >= ch_n[c]) r -= ch_n[c++];
                return ch_lo[c] + r;
            };
            for (int j0 = 0; j0 < n_ang; j0 += per) {
                const int na = min(per, n_ang - j0);
                for (int q = threadIdx.x; q < na * nb; q += blockDim.x) {
                    const int j = q / nb, b = q - j * nb;
                    const TabEntry* Tb = P.tab + (size_t)angle_of(j0 + j) * n_pad + b * kBlock;
                    const int m = min(kBlock, n_pad - b * kBlock);
                    float pw = 0.f, p1 = 0.f;
                    if (staged) {
#pragma unroll 4
                        for (int i = 0; i < m; ++i) {
                            float v, c;
                            vote_fp32<VOTE, HW>(Tb[i], h, staged_at, &v, &c);
                            pw += v;
                            p1 += c;
                        }
                    } else {
                        for (int i = 0; i < m; ++i) {
                            float v, c;
                            vote_fp32<VOTE, HW>(Tb[i], h, gathered_at, &v, &c);
                            pw += v;
                            p1 += c;
                        }
                    }
                    bs_w[q] = pw;
                    bs_1[q] = p1;
                }
                __syncthreads();
                for (int j = threadIdx.x; j < na; j += blockDim.x) {
                    float tw = 0.f, t1 = 0.f;
                    for (int b = 0; b < nb; ++b) {
                        tw += bs_w[j * nb + b];
                        t1 += bs_1[j * nb + b];
                    }
                    const float sw = tw / n_f, s1 = t1 / n_f;
                    const int k = angle_of(j0 + j);
                    if (key_better(sw, s1, 0, 0, k, kw, k1, 0, 0, kk)) {
                        kw = sw;
                        k1 = s1;
                        kk = k;
                    }
                }
                __syncthreads();  // before the next angles' block sums
            }
        }
        // the best of the workgroup by the key (a total order: any merge order gives it)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const float ow = __shfl_xor(kw, off, 64), o1 = __shfl_xor(k1, off, 64);
            const int ok = __shfl_xor(kk, off, 64);
            if (key_better(ow, o1, 0, 0, ok, kw, k1, 0, 0, kk)) {
                kw = ow;
                k1 = o1;
                kk = ok;
            }
        }
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            rw[wv] = kw;
            r1[wv] = k1;
            rk[wv] = kk;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
                if (key_better(rw[w], r1[w], 0, 0, rk[w], kw, k1, 0, 0, kk)) {
                    kw = rw[w];
                    k1 = r1[w];
                    kk = rk[w];
                }
            P.mw[p] = kw;
            P.m1[p] = k1;
            P.mk[p] = kk;
        }
        __syncthreads();  // before the next translation's block and lists
    }
}

constexpr int kCertLds = 64 * 1024;  // largest staged block of k_rescore

// ---------------------------------------------------------------- planning
constexpr int kLC[] = {64, 96, 128, 192, 256};

// Launch-shape knobs of the search kernel: waves stacked in y per workgroup,
// waves splitting the angle chunk, angles per wave, and the window-max form.
// Defaults can be overridden by TM_DENSE_WY / TM_DENSE_WA / TM_DENSE_APW /
// TM_DENSE_ASM (0 to 5: the search kernel variant; tuning runs).
int knob(const char* name, int dflt, int lo, int hi)
{
    const char* v = getenv(name);
    if (!v || !*v) return dflt;
    int x = atoi(v);
    return x < lo ? lo : (x > hi ? hi : x);
}

// d == nullptr: only raise the kernel's LDS limit (done once, before any
// launch, so that no attribute call happens while a stream is captured).
template <int G, int R, int LC, int PREC, int VAR, int VOTE, bool SCREEN>
hipError_t launch_fast_t(const DensePlan& p, const FastArgs& a, const PairDesc* d, int npairs, hipStream_t s)
{
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e =
            hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_fast<G, R, LC, PREC, VAR, VOTE, SCREEN>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (!d) return hipSuccess;
    const dim3 grid = a.work ? dim3(p.n_work) : dim3(p.max_blocks, npairs);
    hipLaunchKernelGGL((k_dense_fast<G, R, LC, PREC, VAR, VOTE, SCREEN>), grid, dim3(64 * p.WY * p.WA), p.lds, s, a,
                       d);
    return hipGetLastError();
}

template <int PREC, int VAR, int VOTE, bool SCREEN>
hipError_t launch_fast_lc(const DensePlan& p, const FastArgs& a, const PairDesc* d, int npairs, hipStream_t s)
{
    switch (p.LC) {
        case 64: return launch_fast_t<32, 8, 64, PREC, VAR, VOTE, SCREEN>(p, a, d, npairs, s);
        case 96: return launch_fast_t<32, 8, 96, PREC, VAR, VOTE, SCREEN>(p, a, d, npairs, s);
        case 128: return launch_fast_t<32, 8, 128, PREC, VAR, VOTE, SCREEN>(p, a, d, npairs, s);
        case 192: return launch_fast_t<32, 8, 192, PREC, VAR, VOTE, SCREEN>(p, a, d, npairs, s);
        default: return launch_fast_t<32, 8, 256, PREC, VAR, VOTE, SCREEN>(p, a, d, npairs, s);
    }
}

// the FP16 screen of a certified detection, or the plain search
template <int PREC, int VAR, int VOTE = 0>
hipError_t launch_fast_p(const DensePlan& p, const FastArgs& a, const PairDesc* d, int npairs, hipStream_t s)
{
    if constexpr (PREC == TM_FP16) {
        if (p.screen) return launch_fast_lc<PREC, VAR, VOTE, true>(p, a, d, npairs, s);
    }
    return launch_fast_lc<PREC, VAR, VOTE, false>(p, a, d, npairs, s);
}

// The edge-taps reading is built in one form per precision, the default one
// (retune_dense offers no other).
constexpr int vote_variant(int precision) { return precision == TM_FP16 ? 4 : 3; }

template <int PREC>
hipError_t launch_fast_v(const DensePlan& p, const FastArgs& a, const PairDesc* d, int npairs, hipStream_t s)
{
    if (p.vote) return launch_fast_p<PREC, vote_variant(PREC), 1>(p, a, d, npairs, s);
    switch (p.variant) {
        case 1: return launch_fast_p<PREC, 1>(p, a, d, npairs, s);
        case 2: return launch_fast_p<PREC, 2>(p, a, d, npairs, s);
        case 3: return launch_fast_p<PREC, 3>(p, a, d, npairs, s);
        case 4: return launch_fast_p<PREC, 4>(p, a, d, npairs, s);
        case 5: return launch_fast_p<PREC, 5>(p, a, d, npairs, s);
        default: return launch_fast_p<PREC, 0>(p, a, d, npairs, s);
    }
}

}  // namespace

void plan_tiles(const DensePlan& p, const PairGeom& g, int* tiles_x, int* tiles_y)
{
    if (!p.fast) {
        *tiles_x = *tiles_y = 0;
        return;
    }
    const int TW = p.G - 2, TH = p.WY * (64 / p.G) * p.R;
    const int Wu = p.tr ? g.H : g.W, Hv = p.tr ? g.W : g.H;  // extents along the lanes and the strips
    *tiles_x = (Wu + TW - 1) / TW;
    *tiles_y = (Hv + TH - 1) / TH;
}

DensePlan plan_dense(const SearchDesc& s, const PairGeom* g, int npairs)
{
    DensePlan p = {};
    p.prec = s.precision;
    p.screen = s.screen && s.precision == TM_FP16;
    int max_halo = 0;
    for (int i = 0; i < npairs; ++i) {
        max_halo = max(max_halo, g[i].rad + 1);
        p.max_rad = max(p.max_rad, g[i].rad);
        p.max_np = max(p.max_np, g[i].gw * g[i].gh);
    }
    p.fast = s.sx == 1 && s.sy == 1 && s.win == 3;
    p.vote = s.vote;
    // measured on the 64-image C2 batch: FP16 fastest with 8 entries per
    // fetch (variant 4), FP32 with 4 (variant 3); all bit-identical to 0
    p.variant = p.vote ? vote_variant(s.precision) : knob("TM_DENSE_ASM", vote_variant(s.precision), 0, 5);
    if (p.fast) {
        p.G = 32;
        p.R = 8;
        p.WY = knob("TM_DENSE_WY", 1, 1, 4);
        p.WA = 4;  // provisional (LDS check); set below with the chunking
        const int TW = p.G - 2, TH = p.WY * (64 / p.G) * p.R;
        p.LC = 0;
        for (int lc : kLC)
            if (lc >= TW + 2 * max_halo) {
                p.LC = lc;
                break;
            }
        // FP16 pixels take 4 bytes (8 with the edge-taps addend), FP32 8
        const size_t px_bytes = s.precision == TM_FP16 ? (p.vote ? 8 : 4) : 8;
        p.tile_lds = (size_t)(TH + 2 * max_halo) * p.LC * px_bytes;
        const size_t comb_bytes = (size_t)(p.screen ? 20 : 12) * p.WA * TH * TW;
        p.lds = p.tile_lds > comb_bytes ? p.tile_lds : comb_bytes;
        if (p.LC == 0 || p.lds > 160 * 1024) p.fast = false;
    }
    if (p.fast) {
        // orientation: the one whose tiles leave fewer translations idle over
        // the whole launch (ties: lanes along x)
        long long cover[2] = {0, 0};
        for (int t = 0; t < 2; ++t) {
            p.tr = t;
            for (int i = 0; i < npairs; ++i) {
                int tx, ty;
                plan_tiles(p, g[i], &tx, &ty);
                cover[t] += (long long)tx * ty;
            }
        }
        p.tr = knob("TM_DENSE_TR", cover[1] < cover[0] ? 1 : 0, 0, 1);
    }
    if (p.fast) {
        // about four waves per SIMD over the whole batch, whole angles per wave
        long long units = 0;
        int max_tiles = 0;
        for (int i = 0; i < npairs; ++i) {
            int tx, ty;
            plan_tiles(p, g[i], &tx, &ty);
            units += (long long)tx * ty * poses_per_translation(s);
            max_tiles = max(max_tiles, tx * ty);
        }
        // fewer (tile, angle) units than four waves per SIMD (a single
        // image): one angle per wave and sixteen waves sharing a tile
        // (measured on one 640x480 FP32 detection: 70.6 us against 73.0 us
        // with four waves, and a quarter of the chunk partials to reduce)
        const bool small = units < 4096;
        long long per_wave = small ? 4 : units / 6144;
        if (per_wave < 1) per_wave = 1;
        per_wave = knob("TM_DENSE_APW", (int)per_wave, 1, 1 << 20);
        // chunks sized for about six waves per SIMD over the batch, then made
        // equal (a multiple of 4 angles each), so that no chunk's workgroups
        // finish far ahead of the others' (measured on the 64-image C2 batch:
        // 360 angles in chunks of 224 + 136, 3.28 ms a launch and 3.02 ms a
        // two-batch step; in 3 of 120, 3.05 ms and 2.88 ms; the autotuner
        // varies the form, not the chunks)
        const int K = poses_per_translation(s);
        p.A = (int)(per_wave * 4);
        p.C = (K + p.A - 1) / p.A;
        p.A = ((K + p.C - 1) / p.C + 3) / 4 * 4;
        p.C = (K + p.A - 1) / p.A;
        p.max_blocks = max_tiles * p.C;
        int wa = knob("TM_DENSE_WA", small ? 16 : 4, 1, 16);
        if (p.WY * wa > 16) wa = 16 / p.WY;
        // a small FP32 launch fetches 8 entries per step too (one 640x480
        // detection: 125.0 against 126.7 us with 4)
        if (small && !p.vote && s.precision == TM_FP32) p.variant = knob("TM_DENSE_ASM", 4, 0, 5);
        if (!retune_dense(p, p.variant, wa)) retune_dense(p, p.variant, 4);
    } else {
        // the generic search reads a copy of the field with a zero border of
        // rad + h + 1 pixels (rad bounds every |q| component)
        p.px_bytes = s.precision == TM_FP16 ? 4 : 8;
        p.win_h = (s.win - 1) / 2;
        for (int i = 0; i < npairs; ++i) {
            const long long pad = g[i].rad + p.win_h + 1;
            p.max_pad_px = max(p.max_pad_px, (long long)(g[i].W + 2 * pad) * (g[i].H + 2 * pad));
        }
        long long np_all = 0;
        for (int i = 0; i < npairs; ++i) np_all += (long long)g[i].gw * g[i].gh;
        const long long blocks = (np_all + 255) / 256;
        long long C = (2048 + blocks - 1) / blocks;  // enough workgroups to fill the chip
        if (C > poses_per_translation(s)) C = poses_per_translation(s);
        if (C < 1) C = 1;
        p.A = (int)((poses_per_translation(s) + C - 1) / C);
        p.C = (poses_per_translation(s) + p.A - 1) / p.A;
    }
    return p;
}

bool retune_dense(DensePlan& p, int variant, int WA)
{
    if (!p.fast || variant < 0 || variant > 5 || WA < 1 || p.WY * WA > 16) return false;
    if (p.vote && variant != p.variant) return false;
    const int TW = p.G - 2, TH = p.WY * (64 / p.G) * p.R;
    const size_t comb_bytes = (size_t)(p.screen ? 20 : 12) * WA * TH * TW;
    const size_t lds = p.tile_lds > comb_bytes ? p.tile_lds : comb_bytes;
    if (lds > 160 * 1024) return false;
    p.variant = variant;
    p.WA = WA;
    p.lds = lds;
    return true;
}

bool rechunk_dense(DensePlan& p, const SearchDesc& s, const PairGeom* g, int npairs, int A)
{
    const int K = poses_per_translation(s);
    if (!p.fast || A < 1) return false;
    A = std::min((A + 3) / 4 * 4, (K + 3) / 4 * 4);  // a multiple of 4 angles, at most all of them
    p.A = A;
    p.C = (K + A - 1) / A;
    int max_tiles = 0;
    for (int i = 0; i < npairs; ++i) {
        int tx, ty;
        plan_tiles(p, g[i], &tx, &ty);
        max_tiles = max(max_tiles, tx * ty);
    }
    p.max_blocks = max_tiles * p.C;
    return true;
}

std::vector<int> chunk_candidates(const DensePlan& p, const SearchDesc& s, int c_max)
{
    std::vector<int> out;
    const int K = poses_per_translation(s);
    if (!p.fast) return out;
    for (int C = 1; C <= c_max; ++C) {
        const int A = std::min(((K + C - 1) / C + 3) / 4 * 4, (K + 3) / 4 * 4);
        if ((K + A - 1) / A <= c_max && std::find(out.begin(), out.end(), A) == out.end()) out.push_back(A);
    }
    return out;
}

bool build_work(const DensePlan& p, const PairGeom* g, int npairs, std::vector<int2>& out)
{
    out.clear();
    if (!p.fast || !knob("TM_DENSE_WORKLIST", 1, 0, 1)) return true;
    constexpr int kXcd = 8;
    struct Run {
        int pair, blocks;
        double cost;  // per block: its points (the taps scale with n) plus the tile staging
    };
    std::vector<Run> runs;
    double total = 0;
    for (int i = 0; i < npairs; ++i) {
        int tx, ty;
        plan_tiles(p, g[i], &tx, &ty);
        const Run r{i, tx * ty * p.C, (double)g[i].n + 8.0};
        runs.push_back(r);
        total += r.cost * r.blocks;
    }
    std::stable_sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) { return a.cost > b.cost; });
    // Fill the bins in turn, heaviest blocks first, each to an equal share of
    // the cost; a pair's blocks stay contiguous (split over at most a few bins).
    std::vector<std::vector<int2>> bin(kXcd);
    const double share = total / kXcd;
    int b = 0;
    double load = 0;
    for (const Run& r : runs)
        for (int k = 0; k < r.blocks; ++k) {
            if (load >= share && b < kXcd - 1) {
                ++b;
                load = 0;
            }
            bin[b].push_back(make_int2(r.pair, k));
            load += r.cost;
        }
    size_t longest = 0;
    for (auto& v : bin) longest = std::max(longest, v.size());
    // Workgroup w is dispatched to XCD w % 8: interleave the bins.
    out.assign(longest * kXcd, make_int2(-1, 0));
    for (int x = 0; x < kXcd; ++x)
        for (size_t j = 0; j < bin[x].size(); ++j) out[j * kXcd + x] = bin[x][j];
    // every block of every pair exactly once
    std::vector<int> first(npairs + 1, 0);
    for (const Run& r : runs) first[r.pair + 1] = r.blocks;
    for (int i = 0; i < npairs; ++i) first[i + 1] += first[i];
    std::vector<unsigned char> seen(first[npairs], 0);
    for (const int2& w : out) {
        if (w.x < 0) continue;
        if (w.x >= npairs || w.y < 0 || w.y >= first[w.x + 1] - first[w.x] || seen[first[w.x] + w.y]++) return false;
    }
    for (unsigned char c : seen)
        if (!c) return false;
    return true;
}

size_t dense_partials_bytes(const DensePlan& p, int np) { return (size_t)p.C * np * (p.screen ? 24 : 12); }

hipError_t prepare_dense(const SearchDesc& s, const DensePlan& p)
{
    if (!p.fast) return hipSuccess;
    FastArgs a = {};
    if (s.precision == TM_FP16)
        return launch_fast_v<TM_FP16>(p, a, nullptr, 0, nullptr);
    return launch_fast_v<TM_FP32>(p, a, nullptr, 0, nullptr);
}

hipError_t launch_dense(const SearchDesc& s, const DensePlan& p, const PairDesc* d, int npairs, hipStream_t st,
                        hipEvent_t ev0, hipEvent_t ev1, int* cert_count)
{
    hipError_t e;
    if (ev0) {
        e = hipEventRecord(ev0, st);
        if (e != hipSuccess) return e;
    }
    if (p.fast) {
        FastArgs a;
        a.level = s.level;
        a.tr = p.tr;
        a.K = poses_per_translation(s);
        a.A = p.A;
        a.WY = p.WY;
        a.WA = p.WA;
        a.C = p.C;
        a.work = p.work;
        if (s.precision == TM_FP16)
            e = launch_fast_v<TM_FP16>(p, a, d, npairs, st);
        else
            e = launch_fast_v<TM_FP32>(p, a, d, npairs, st);
    } else {
        GenericArgs a;
        a.level = s.level;
        a.K = poses_per_translation(s);
        a.A = p.A;
        a.sx = s.sx;
        a.sy = s.sy;
        a.win = s.win;
        const dim3 pgrid((unsigned)((p.max_pad_px + 255) / 256), npairs);
        if (s.precision == TM_FP16)
            hipLaunchKernelGGL(k_pad_field<TM_FP16>, pgrid, dim3(256), 0, st, s.level, d);
        else
            hipLaunchKernelGGL(k_pad_field<TM_FP32>, pgrid, dim3(256), 0, st, s.level, d);
        dim3 grid((p.max_np + 255) / 256, p.C, npairs);
        if (s.precision == TM_FP16 && p.screen) {
            if (s.vote)
                hipLaunchKernelGGL((k_dense_generic<TM_FP16, 1, true>), grid, dim3(256), 0, st, a, d);
            else
                hipLaunchKernelGGL((k_dense_generic<TM_FP16, 0, true>), grid, dim3(256), 0, st, a, d);
        } else if (s.precision == TM_FP16) {
            if (s.vote)
                hipLaunchKernelGGL((k_dense_generic<TM_FP16, 1>), grid, dim3(256), 0, st, a, d);
            else
                hipLaunchKernelGGL((k_dense_generic<TM_FP16, 0>), grid, dim3(256), 0, st, a, d);
        } else {
            if (s.vote)
                hipLaunchKernelGGL((k_dense_generic<TM_FP32, 1>), grid, dim3(256), 0, st, a, d);
            else
                hipLaunchKernelGGL((k_dense_generic<TM_FP32, 0>), grid, dim3(256), 0, st, a, d);
        }
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (ev1) {
        e = hipEventRecord(ev1, st);
        if (e != hipSuccess) return e;
    }
    if (p.screen)
        hipLaunchKernelGGL(k_reduce_screen, dim3((p.max_np + 255) / 256, npairs), dim3(256), 0, st, p.C, d,
                           cert_count);
    else
        hipLaunchKernelGGL(k_reduce_chunks, dim3((p.max_np + kRedPos - 1) / kRedPos, npairs),
                           dim3(kRedPos * kRedLanes), 0, st, p.C, d);
    return hipGetLastError();
}

template <int PREC, int VOTE>
void launch_sparse_t(const void* field, int W, int H, const ModelPoint* pts, int n, int win, const tm_eval_pose* poses,
                     int np, float* scores, hipStream_t s)
{
    hipLaunchKernelGGL((k_sparse<PREC, VOTE>), dim3((np + 3) / 4), dim3(256), 0, s, field, W, H, pts, n, win, poses,
                       np, scores);
}

hipError_t launch_sparse(const void* field, int W, int H, int precision, const ModelPoint* pts, int n, int win,
                         int vote, const tm_eval_pose* poses, int np, float* scores, hipStream_t s)
{
    if (np == 0) return hipSuccess;
    if (precision == TM_FP16) {
        if (vote)
            launch_sparse_t<TM_FP16, 1>(field, W, H, pts, n, win, poses, np, scores, s);
        else
            launch_sparse_t<TM_FP16, 0>(field, W, H, pts, n, win, poses, np, scores, s);
    } else {
        if (vote)
            launch_sparse_t<TM_FP32, 1>(field, W, H, pts, n, win, poses, np, scores, s);
        else
            launch_sparse_t<TM_FP32, 0>(field, W, H, pts, n, win, poses, np, scores, s);
    }
    return hipGetLastError();
}

size_t cert_bytes(int total_np) { return 256 + (size_t)total_np * sizeof(int4) + 256; }

CertBufs cert_bufs(void* base, int total_np)
{
    CertBufs b;
    uint8_t* q = reinterpret_cast<uint8_t*>(base);
    b.count = reinterpret_cast<int*>(q);
    b.list = reinterpret_cast<int4*>(q + 256);
    b.cap = total_np;
    return b;
}

namespace {
template <int VOTE, int HW>
hipError_t rescore_attr()
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rescore<VOTE, HW>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kCertLds);
}
}  // namespace

hipError_t launch_certify(const SearchDesc& s, const DensePlan& p, const PairDesc* d, int npairs, const CertBufs& cb,
                          hipStream_t st, bool count_cleared)
{
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = rescore_attr<0, 1>();
        if (e == hipSuccess) e = rescore_attr<1, 1>();
        if (e == hipSuccess) e = rescore_attr<0, -1>();
        if (e == hipSuccess) e = rescore_attr<1, -1>();
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (!d) return hipSuccess;
    CertArgs a;
    a.level = s.level;
    a.C = p.C;
    a.A = p.A;
    a.K = poses_per_translation(s);
    a.win = s.win;
    a.sx = s.sx;
    a.sy = s.sy;
    a.min_score = s.min_score;
    a.cb = cb;
    // pairs whose block fits are staged, larger ones gather from memory
    const int B = p.max_rad + (s.win - 1) / 2, S = 2 * B + 1;
    a.lds_bytes = (long long)S * S * 8 <= kCertLds ? S * S * 8 : kCertLds;
    if (!count_cleared) hipLaunchKernelGGL(k_cert_zero, dim3(1), dim3(64), 0, st, cb.count);
    hipLaunchKernelGGL(k_certify, dim3((p.max_np + 255) / 256, npairs), dim3(256), 0, st, a, d);
    const dim3 grid(min(cb.cap, 4096)), block(256);
    if (s.win == 3) {
        if (s.vote)
            hipLaunchKernelGGL((k_rescore<1, 1>), grid, block, a.lds_bytes, st, a, d);
        else
            hipLaunchKernelGGL((k_rescore<0, 1>), grid, block, a.lds_bytes, st, a, d);
    } else {
        if (s.vote)
            hipLaunchKernelGGL((k_rescore<1, -1>), grid, block, a.lds_bytes, st, a, d);
        else
            hipLaunchKernelGGL((k_rescore<0, -1>), grid, block, a.lds_bytes, st, a, d);
    }
    return hipGetLastError();
}

}  // namespace tmk
