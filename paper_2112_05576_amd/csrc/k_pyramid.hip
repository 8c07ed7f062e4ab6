// Edge extraction and image pyramid (Sec. II para. 2): uint8 levels by 2x2
// rounded means, integer Sobel gradients, magnitude threshold and unit
// gradient directions per level; model edge points in row-major order.
#include "tm_device.h"

namespace tmk {

namespace {


// One workgroup takes a 64x64 block of level `base` and produces the matching
// cells of levels base+1 .. top (at most 6 more levels: 32x32 down to 1x1).
// Every output pixel depends only on its own 2^k x 2^k block, so blocks are
// independent.  Level `base` is read from `src` (pitched); when base == 0 the
// block is also copied into level 0.
template <bool BATCH>
__global__ __launch_bounds__(256) void k_pyr_build(PyrBuildArg one, const PyrBuildArg* __restrict__ many, int base,
                                                    int top, int copy_base)
{
    __shared__ uint8_t cells[16 * 16];
    const uint3 B = xcd_block();  // (block column, block row, image)
    const PyrBuildArg& lv = BATCH ? many[B.z] : one;
    top = min(top, lv.L - 1);
    if ((int)B.x * 64 >= lv.w[base] || (int)B.y * 64 >= lv.h[base]) return;
    const uint8_t* __restrict__ src = base == 0 ? lv.src : lv.img[base];
    const int src_pitch = base == 0 ? lv.pitch : lv.w[base];
    const int t = threadIdx.x;
    const int cx = t & 15, cy = t >> 4;
    const int W = lv.w[base], H = lv.h[base];
    const int x0 = B.x * 64 + cx * 4;
    const int y0 = B.y * 64 + cy * 4;
    int v[4][4];
    // a row's four bytes as one word where they are whole and aligned
    const bool words = x0 + 3 < W && ((reinterpret_cast<uintptr_t>(src) | (uintptr_t)src_pitch) & 3) == 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int y = y0 + j;
        if (words) {
            const uint32_t w = y < H ? *reinterpret_cast<const uint32_t*>(src + (size_t)y * src_pitch + x0) : 0u;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[j][i] = (int)((w >> (8 * i)) & 0xffu);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = x0 + i;
                v[j][i] = (x < W && y < H) ? (int)src[(size_t)y * src_pitch + x] : 0;
            }
        }
    }
    if (copy_base) {
        uint8_t* dst = lv.img[base];
        const bool wdst = words && (W & 3) == 0 && (reinterpret_cast<uintptr_t>(dst) & 3) == 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (y0 + j >= H) continue;
            if (wdst) {
                *reinterpret_cast<uint32_t*>(dst + (size_t)(y0 + j) * W + x0) =
                    (uint32_t)v[j][0] | ((uint32_t)v[j][1] << 8) | ((uint32_t)v[j][2] << 16) | ((uint32_t)v[j][3] << 24);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (x0 + i < W) dst[(size_t)(y0 + j) * W + x0 + i] = (uint8_t)v[j][i];
            }
        }
    }
    if (top <= base) return;
    // level base+1: a 2x2 patch per thread
    int l1[2][2];
    {
        const int l = base + 1, W1 = lv.w[l], H1 = lv.h[l];
        const int bx = B.x * 32 + cx * 2, by = B.y * 32 + cy * 2;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                int s = v[2 * j][2 * i] + v[2 * j][2 * i + 1] + v[2 * j + 1][2 * i] + v[2 * j + 1][2 * i + 1];
                l1[j][i] = (s + 2) >> 2;
                if (bx + i < W1 && by + j < H1) lv.img[l][(size_t)(by + j) * W1 + bx + i] = (uint8_t)l1[j][i];
            }
    }
    if (top <= base + 1) return;
    // level base+2: one pixel per thread, kept in LDS for the levels above
    {
        const int l = base + 2, W2 = lv.w[l], H2 = lv.h[l];
        int s = l1[0][0] + l1[0][1] + l1[1][0] + l1[1][1];
        int p = (s + 2) >> 2;
        int x = B.x * 16 + cx, y = B.y * 16 + cy;
        if (x < W2 && y < H2) lv.img[l][(size_t)y * W2 + x] = (uint8_t)p;
        cells[cy * 16 + cx] = (uint8_t)p;
    }
    int side = 16;
    for (int l = base + 3; l <= top && l <= base + 6; ++l) {
        __syncthreads();
        const int ns = side / 2;
        int p = 0;
        const bool act = t < ns * ns;
        const int ix = t % ns, iy = t / ns;
        if (act) {
            int s = cells[(2 * iy) * side + 2 * ix] + cells[(2 * iy) * side + 2 * ix + 1] +
                    cells[(2 * iy + 1) * side + 2 * ix] + cells[(2 * iy + 1) * side + 2 * ix + 1];
            p = (s + 2) >> 2;
            const int Wl = lv.w[l], Hl = lv.h[l];
            int x = B.x * ns + ix, y = B.y * ns + iy;
            if (x < Wl && y < Hl) lv.img[l][(size_t)y * Wl + x] = (uint8_t)p;
        }
        __syncthreads();
        if (act) cells[iy * ns + ix] = (uint8_t)p;
        side = ns;
    }
}


__device__ __forceinline__ void sobel_at(const uint8_t* __restrict__ img, int W, int H, int x, int y, int* gx,
                                         int* gy)
{
    if (x < 1 || y < 1 || x > W - 2 || y > H - 2) {
        *gx = 0;
        *gy = 0;
        return;
    }
    const uint8_t* r0 = img + (size_t)(y - 1) * W + x;
    const uint8_t* r1 = r0 + W;
    const uint8_t* r2 = r1 + W;
    int a = r0[-1], b = r0[0], c = r0[1];
    int d = r1[-1], f = r1[1];
    int g = r2[-1], h = r2[0], i = r2[1];
    *gx = (c + 2 * f + i) - (a + 2 * d + g);
    *gy = (g + 2 * h + i) - (a + 2 * b + c);
}

__device__ __forceinline__ uint32_t pack_grad(int gx, int gy)
{
    return (uint32_t)(uint16_t)(int16_t)gx | ((uint32_t)(uint16_t)(int16_t)gy << 16);
}

__device__ __forceinline__ void unpack_grad(uint32_t v, int* gx, int* gy)
{
    *gx = (int)(int16_t)(v & 0xFFFFu);
    *gy = (int)(int16_t)(v >> 16);
}

// The gradient pair of a pixel of level l: read from the gradient-map pyramid
// where there is one, else the Sobel pair of the level's image.
__device__ __forceinline__ void level_grad(const uint8_t* img, const uint32_t* grad, int W, int H, int x, int y,
                                           int* gx, int* gy)
{
    if (grad)
        unpack_grad(grad[(size_t)y * W + x], gx, gy);
    else
        sobel_at(img, W, H, x, y, gx, gy);
}

// One level of the gradient-map pyramid, one thread per pixel: level 0 is the
// Sobel pair of the full image; level l > 0 takes the 2x2 block of level l-1
// and floors (s + 2) / 4 per component (an arithmetic shift by 2 is a floored
// division of the signed sum).  Components stay within the Sobel range
// |g| <= 1020, so they pack as int16.  grid: (pixels / 256, image).
template <bool BATCH>
__global__ __launch_bounds__(256) void k_grad_level(FieldsArg one, const FieldsArg* __restrict__ many, int l)
{
    const FieldsArg& a = BATCH ? many[blockIdx.y] : one;
    if (l >= a.L) return;
    const int W = a.w[l], H = a.h[l];
    const int idx = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (idx >= W * H) return;
    const int y = idx / W, x = idx - y * W;
    int gx, gy;
    if (l == 0) {
        sobel_at(a.img[0], W, H, x, y, &gx, &gy);
    } else {
        const int Wp = a.w[l - 1];
        const uint32_t* __restrict__ src = a.grad[l - 1] + (size_t)(2 * y) * Wp + 2 * x;
        int sx = 0, sy = 0;
        const uint32_t v[4] = {src[0], src[1], src[Wp], src[Wp + 1]};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int u, w;
            unpack_grad(v[j], &u, &w);
            sx += u;
            sy += w;
        }
        gx = (sx + 2) >> 2;
        gy = (sy + 2) >> 2;
    }
    a.grad[l][idx] = pack_grad(gx, gy);
}

// (gx, gy)/|g| rounded to FP32, for |gx|, |gy| <= 1020 (the Sobel range, which
// the gradient-map levels keep) and m2 = gx^2 + gy^2 > 0.  1/|g| is the FP32
// reciprocal square root (relative error within 2^-22) refined by two Newton
// steps in FP64, each of which squares the error (it ends below 2^-50); the
// products gx/|g|, gy/|g| are formed in FP64 and rounded once.  Over that
// range every quotient lies at least 2^-43.9 (relative) from the midpoint of
// two FP32 neighbours (found by enumerating all pairs), so the result is the
// FP32 rounding of the exact quotient: the bits FP64 square root and division
// give, with no FP64 division and no FP64 square root.
__device__ __forceinline__ void unit_dir(int gx, int gy, int m2, float* fx, float* fy)
{
    const double md = (double)m2;
    double r = (double)__builtin_amdgcn_rsqf((float)m2);  // m2 <= 2 * 1020^2 is exact in FP32
    r = fma(0.5 * r, fma(-md * r, r, 1.0), r);
    r = fma(0.5 * r, fma(-md * r, r, 1.0), r);
    *fx = (float)((double)gx * r);
    *fy = (float)((double)gy * r);
}

// Unit gradient direction of every pixel of every level: (gx, gy)/|g| rounded
// once to the storage precision where gx^2 + gy^2 > T2, (0, 0) elsewhere (an
// FP16 pyramid also gets the FP32 rounding, its twin).  Each thread covers 4
// consecutive pixels of a row; their 3 x 6 neighbourhood (three aligned words
// per row where rows start on a word, else bytes; or their 4 gradient pairs)
// is loaded at once, before any of the four is computed, so a thread waits
// for memory once.
template <bool BATCH>
__global__ __launch_bounds__(256) void k_sobel_fields(FieldsArg one, const FieldsArg* __restrict__ many)
{
    const uint3 B = xcd_block();  // (block, image)
    const FieldsArg& a = BATCH ? many[B.y] : one;
    if ((int)B.x >= a.block0[a.L]) return;
    const long long T2 = a.T2;
    const int precision = a.precision;
    int l = 0;
    while (l + 1 < a.L && (int)B.x >= a.block0[l + 1]) ++l;
    const int W = a.w[l], H = a.h[l];
    const int qw = (W + 3) / 4;
    const int idx = ((int)B.x - a.block0[l]) * 256 + (int)threadIdx.x;
    const int y = idx / qw, x0 = (idx % qw) * 4;
    if (y >= H) return;
    const uint8_t* __restrict__ img = a.img[l];
    const uint32_t* __restrict__ grad = a.grad[l];
    int gxv[4], gyv[4];
    if (grad) {
        uint32_t v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = grad[(size_t)y * W + min(x0 + i, W - 1)];
#pragma unroll
        for (int i = 0; i < 4; ++i) unpack_grad(v[i], &gxv[i], &gyv[i]);
    } else {
        // rows y-1 .. y+1, columns x0-1 .. x0+4, at clamped addresses: a
        // clamped value only ever feeds a pixel of the one-pixel frame,
        // whose gradient is 0
        int p[3][6];
        if ((W & 3) == 0 && (reinterpret_cast<uintptr_t>(img) & 3) == 0) {
            // words x0/4 - 1 .. x0/4 + 1 of each row, clamped to the row (a
            // clamped word only feeds the frame as above)
            const int q = x0 >> 2, nq = W >> 2;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const uint32_t* rw =
                    reinterpret_cast<const uint32_t*>(img + (size_t)min(max(y - 1 + r, 0), H - 1) * W);
                const uint32_t wl = rw[max(q - 1, 0)], wc = rw[q], wr = rw[min(q + 1, nq - 1)];
                p[r][0] = (int)(wl >> 24);
#pragma unroll
                for (int c = 0; c < 4; ++c) p[r][1 + c] = (int)((wc >> (8 * c)) & 0xFFu);
                p[r][5] = (int)(wr & 0xFFu);
            }
        } else {
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const size_t row = (size_t)min(max(y - 1 + r, 0), H - 1) * W;
#pragma unroll
                for (int c = 0; c < 6; ++c) p[r][c] = img[row + min(max(x0 - 1 + c, 0), W - 1)];
            }
        }
        const bool row_in = y >= 1 && y <= H - 2;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = x0 + i;
            const bool in = row_in && x >= 1 && x <= W - 2;
            const int gx = (p[0][i + 2] + 2 * p[1][i + 2] + p[2][i + 2]) - (p[0][i] + 2 * p[1][i] + p[2][i]);
            const int gy = (p[2][i] + 2 * p[2][i + 1] + p[2][i + 2]) - (p[0][i] + 2 * p[0][i + 1] + p[0][i + 2]);
            gxv[i] = in ? gx : 0;
            gyv[i] = in ? gy : 0;
        }
    }
    float fx[4], fy[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gx = gxv[i], gy = gyv[i];
        const long long m2 = (long long)gx * gx + (long long)gy * gy;
        fx[i] = 0.0f;
        fy[i] = 0.0f;
        if (m2 > T2 && m2 > 0) unit_dir(gx, gy, (int)m2, &fx[i], &fy[i]);
    }
    const size_t o = (size_t)y * W + x0;
    // FP32 pairs: two pixels per 16-byte store where the four are whole and
    // the row offset keeps the alignment
    float* f32 = reinterpret_cast<float*>(precision == TM_FP16 ? a.field32[l] : a.field[l]);
    if (f32) {
        if (x0 + 3 < W && (o & 1) == 0) {
            float4* q = reinterpret_cast<float4*>(f32 + 2 * o);
            q[0] = make_float4(fx[0], fy[0], fx[1], fy[1]);
            q[1] = make_float4(fx[2], fy[2], fx[3], fy[3]);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (x0 + i < W) reinterpret_cast<float2*>(f32)[o + i] = make_float2(fx[i], fy[i]);
        }
    }
    // the FP16 field (a batch's pyramid keeps it at its searched level only);
    // an FP16 pyramid's FP32 pairs above are the twin its decisions read
    if (precision == TM_FP16 && a.field[l]) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (x0 + i < W) reinterpret_cast<__half2*>(a.field[l])[o + i] = __floats2half2_rn(fx[i], fy[i]);
    }
}

struct PointsArg {
    const uint8_t* img[kMaxLevels];
    const uint32_t* grad[kMaxLevels];  // gradient-map pyramid, or null
    ModelPoint* pts[kMaxLevels];
    int w[kMaxLevels];
    int h[kMaxLevels];
    int* counts;
};

// One workgroup per model level: thread t scans a contiguous run of pixels,
// counts its edge pixels, an exclusive scan gives each run its output offset,
// and a second pass writes the points, so the list is in row-major order.
__global__ __launch_bounds__(1024) void k_model_points(PointsArg a, long long T2)
{
    __shared__ int scan[1024];
    const int l = blockIdx.x;
    const int W = a.w[l], H = a.h[l];
    const int N = W * H;
    const int per = (N + 1023) / 1024;
    const int p0 = min(N, (int)threadIdx.x * per), p1 = min(N, p0 + per);
    const uint8_t* img = a.img[l];
    const uint32_t* grad = a.grad[l];
    int cnt = 0;
    for (int p = p0; p < p1; ++p) {
        int gx, gy;
        level_grad(img, grad, W, H, p % W, p / W, &gx, &gy);
        cnt += ((long long)gx * gx + (long long)gy * gy > T2) ? 1 : 0;
    }
    scan[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
        int v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    int o = scan[threadIdx.x] - cnt;
    const int cx = W / 2, cy = H / 2;
    for (int p = p0; p < p1; ++p) {
        int x = p % W, y = p / W, gx, gy;
        level_grad(img, grad, W, H, x, y, &gx, &gy);
        if ((long long)gx * gx + (long long)gy * gy > T2) {
            ModelPoint mp;
            mp.tx = (int16_t)(x - cx);
            mp.ty = (int16_t)(y - cy);
            mp.gx = (int16_t)gx;
            mp.gy = (int16_t)gy;
            a.pts[l][o++] = mp;
        }
    }
    if (threadIdx.x == 1023) a.counts[l] = scan[1023];
}

}  // namespace

PyrBuildArg pyr_build_arg(const uint8_t* src, int src_pitch, const PyrLevel* lv, int L)
{
    PyrBuildArg a = {};
    a.src = src;
    a.pitch = src_pitch;
    a.L = L;
    for (int l = 0; l < L; ++l) {
        a.img[l] = lv[l].img;
        a.w[l] = lv[l].w;
        a.h[l] = lv[l].h;
    }
    return a;
}

FieldsArg fields_arg(const PyrLevel* lv, int L, long long T2, int precision)
{
    FieldsArg a = {};
    a.L = L;
    a.T2 = T2;
    a.precision = precision;
    int blocks = 0;
    for (int l = 0; l < L; ++l) {
        a.img[l] = lv[l].img;
        a.grad[l] = lv[l].grad;
        a.field[l] = lv[l].field;
        a.field32[l] = precision == TM_FP16 ? lv[l].field32 : nullptr;
        a.w[l] = lv[l].w;
        a.h[l] = lv[l].h;
        a.block0[l] = blocks;
        long long quads = (long long)((lv[l].w + 3) / 4) * lv[l].h;
        blocks += (int)((quads + 255) / 256);
    }
    a.block0[L] = blocks;
    return a;
}

// Level passes: levels 1..6 from the caller's image, then (more than 7
// levels) from the last level produced.
hipError_t launch_pyr_build(const uint8_t* src, int src_pitch, const PyrLevel* lv, int L, hipStream_t s)
{
    PyrBuildArg a = pyr_build_arg(src, src_pitch, lv, L);
    for (int base = 0;; base += 6) {
        const int top = min(L - 1, base + 6);
        dim3 grid((a.w[base] + 63) / 64, (a.h[base] + 63) / 64);
        hipLaunchKernelGGL(k_pyr_build<false>, grid, dim3(256), 0, s, a, nullptr, base, top, base == 0 ? 1 : 0);
        if (top >= L - 1) break;
    }
    return hipGetLastError();
}

hipError_t launch_grad_pyramid(const PyrLevel* lv, int L, hipStream_t s)
{
    FieldsArg a = fields_arg(lv, L, 0, TM_FP32);
    for (int l = 0; l < L; ++l) {
        if (!a.grad[l]) return hipErrorInvalidValue;
        const long long px = (long long)a.w[l] * a.h[l];
        hipLaunchKernelGGL(k_grad_level<false>, dim3((unsigned)((px + 255) / 256)), dim3(256), 0, s, a, nullptr, l);
    }
    return hipGetLastError();
}

hipError_t launch_sobel_fields(const PyrLevel* lv, int L, long long T2, int precision, hipStream_t s)
{
    FieldsArg a = fields_arg(lv, L, T2, precision);
    hipLaunchKernelGGL(k_sobel_fields<false>, dim3(a.block0[L]), dim3(256), 0, s, a, nullptr);
    return hipGetLastError();
}

hipError_t launch_pyramids_batch(const PyrBuildArg* pb, const FieldsArg* fa, int n_images, int L, int max_w,
                                 int max_h, int max_field_blocks, const int* level_w, const int* level_h,
                                 bool gradient, hipStream_t s)
{
    for (int base = 0;; base += 6) {
        const int top = min(L - 1, base + 6);
        dim3 grid((level_w[base] + 63) / 64, (level_h[base] + 63) / 64, n_images);
        hipLaunchKernelGGL(k_pyr_build<true>, grid, dim3(256), 0, s, PyrBuildArg{}, pb, base, top,
                           base == 0 ? 1 : 0);
        if (top >= L - 1) break;
    }
    (void)max_w;
    (void)max_h;
    // level_w x level_h bounds every image's level; the kernel checks its own size
    for (int l = 0; gradient && l < L; ++l) {
        const long long px = (long long)level_w[l] * level_h[l];
        hipLaunchKernelGGL(k_grad_level<true>, dim3((unsigned)((px + 255) / 256), n_images), dim3(256), 0, s,
                           FieldsArg{}, fa, l);
    }
    hipLaunchKernelGGL(k_sobel_fields<true>, dim3(max_field_blocks, n_images), dim3(256), 0, s, FieldsArg{}, fa);
    return hipGetLastError();
}

hipError_t launch_model_points(const PyrLevel* lv, int L, long long T2, ModelPoint* const* pts, int* counts,
                               hipStream_t s)
{
    PointsArg a = {};
    for (int l = 0; l < L; ++l) {
        a.img[l] = lv[l].img;
        a.grad[l] = lv[l].grad;
        a.pts[l] = pts[l];
        a.w[l] = lv[l].w;
        a.h[l] = lv[l].h;
    }
    a.counts = counts;
    hipLaunchKernelGGL(k_model_points, dim3(L), dim3(1024), 0, s, a, T2);
    return hipGetLastError();
}

}  // namespace tmk
