// Ceiling probes for the roofline of the search kernel (measurement, not the
// method): kernels that run one instruction mix of the exhaustive search at
// full occupancy and nothing else, so that their rates are what the hardware
// achieves for that mix.  The caller times a launch; the work it enqueued is
// returned so that the rate needs no instruction counting outside.
//  * VALU mix: per iteration and wave, the search kernel's arithmetic for one
//    model point and an 8-row strip (written out in assembly, so the count is
//    exact): 10 v_dot2_f32_f16, 8 v_max3_f32, 16 v_max_f32 with a DPP wave
//    shift, 8 v_add_f32 (the windowed sums); 42 VALU instructions.
//  * VALU adds: 32 independent v_add_f32 per iteration (the plain issue rate),
//    and one class at a time: v_dot2_f32_f16, DPP v_max_f32, v_max3_f32.
//  * LDS: the search kernel's tile reads for one point: 10 rows of a strip,
//    one 4-byte pixel per lane per row, rows 64 words apart, at an offset
//    that changes every iteration (as the rotated point offsets do).
//  * HBM: a streaming copy of one half of a buffer into the other (16-byte
//    loads and stores, every byte read once and written once).
#include "tm_internal.h"

namespace tmk {

namespace {

constexpr int kProbeThreads = 256;

// The search kernel's per-point arithmetic, written out: ten products of a
// half2 direction with ten half2 field values (FP32 results), the vertical
// maxima of three, the horizontal maxima through wave-shift DPP, the sums.
// Hazards as in the search kernel: three wait states after a dot before its
// result is read (s_nop 2), two after a VALU write before a DPP read of it
// (s_nop 1).
__global__ __launch_bounds__(kProbeThreads) void k_probe_valu_mix(int iters, float* out)
{
    uint32_t g[10];
    const uint32_t seed = (uint32_t)(threadIdx.x * 2654435761u) ^ blockIdx.x;
#pragma unroll
    for (int j = 0; j < 10; ++j) g[j] = (seed + 0x3c003c00u * (uint32_t)j) & 0x3bff3bffu;  // half2 below 1
    const uint32_t rh = 0x39a839a8u;  // half2 (0.707, 0.707)
    float acc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = 0.f;
    for (int it = 0; it < iters; ++it) {
        float d[10], v[8], m[8];
        asm volatile(
            "v_dot2_f32_f16 %0, %10, %11, 0\n\t"
            "v_dot2_f32_f16 %1, %10, %12, 0\n\t"
            "v_dot2_f32_f16 %2, %10, %13, 0\n\t"
            "v_dot2_f32_f16 %3, %10, %14, 0\n\t"
            "v_dot2_f32_f16 %4, %10, %15, 0\n\t"
            "v_dot2_f32_f16 %5, %10, %16, 0\n\t"
            "v_dot2_f32_f16 %6, %10, %17, 0\n\t"
            "v_dot2_f32_f16 %7, %10, %18, 0\n\t"
            "v_dot2_f32_f16 %8, %10, %19, 0\n\t"
            "v_dot2_f32_f16 %9, %10, %20, 0\n\t"
            "s_nop 2"
            : "=&v"(d[0]), "=&v"(d[1]), "=&v"(d[2]), "=&v"(d[3]), "=&v"(d[4]), "=&v"(d[5]), "=&v"(d[6]),
              "=&v"(d[7]), "=&v"(d[8]), "=&v"(d[9])
            : "s"(rh), "v"(g[0]), "v"(g[1]), "v"(g[2]), "v"(g[3]), "v"(g[4]), "v"(g[5]), "v"(g[6]), "v"(g[7]),
              "v"(g[8]), "v"(g[9]));
        asm volatile(
            "v_max3_f32 %0, %8, %9, %10\n\t"
            "v_max3_f32 %1, %9, %10, %11\n\t"
            "v_max3_f32 %2, %10, %11, %12\n\t"
            "v_max3_f32 %3, %11, %12, %13\n\t"
            "v_max3_f32 %4, %12, %13, %14\n\t"
            "v_max3_f32 %5, %13, %14, %15\n\t"
            "v_max3_f32 %6, %14, %15, %16\n\t"
            "v_max3_f32 %7, %15, %16, %17\n\t"
            "s_nop 1"
            : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]), "=&v"(v[6]),
              "=&v"(v[7])
            : "v"(d[0]), "v"(d[1]), "v"(d[2]), "v"(d[3]), "v"(d[4]), "v"(d[5]), "v"(d[6]), "v"(d[7]), "v"(d[8]),
              "v"(d[9]));
        asm volatile(
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
            : "=&v"(m[0]), "=&v"(m[1]), "=&v"(m[2]), "=&v"(m[3]), "=&v"(m[4]), "=&v"(m[5]), "=&v"(m[6]),
              "=&v"(m[7])
            : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]));
        asm volatile(
            "v_add_f32 %0, %0, %8\n\t"
            "v_add_f32 %1, %1, %9\n\t"
            "v_add_f32 %2, %2, %10\n\t"
            "v_add_f32 %3, %3, %11\n\t"
            "v_add_f32 %4, %4, %12\n\t"
            "v_add_f32 %5, %5, %13\n\t"
            "v_add_f32 %6, %6, %14\n\t"
            "v_add_f32 %7, %7, %15"
            : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]), "+v"(acc[6]),
              "+v"(acc[7])
            : "v"(m[0]), "v"(m[1]), "v"(m[2]), "v"(m[3]), "v"(m[4]), "v"(m[5]), "v"(m[6]), "v"(m[7]));
    }
    float t = 0.f;
#pragma unroll
    for (int r = 0; r < 8; ++r) t += acc[r];
    if (t == 12345.f) out[0] = t;  // keeps the loop; never true for these inputs
}
constexpr int kMixValu = 42;  // VALU instructions per iteration of k_probe_valu_mix

__global__ __launch_bounds__(kProbeThreads) void k_probe_valu_add(int iters, float* out)
{
    float a[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) a[j] = (float)(threadIdx.x + j);
    const float b = 1.0e-7f * (float)(blockIdx.x + 1);
    for (int it = 0; it < iters; ++it) {
        asm volatile(
            "v_add_f32 %0, %0, %32\n\tv_add_f32 %1, %1, %32\n\tv_add_f32 %2, %2, %32\n\tv_add_f32 %3, %3, %32\n\t"
            "v_add_f32 %4, %4, %32\n\tv_add_f32 %5, %5, %32\n\tv_add_f32 %6, %6, %32\n\tv_add_f32 %7, %7, %32\n\t"
            "v_add_f32 %8, %8, %32\n\tv_add_f32 %9, %9, %32\n\tv_add_f32 %10, %10, %32\n\tv_add_f32 %11, %11, %32\n\t"
            "v_add_f32 %12, %12, %32\n\tv_add_f32 %13, %13, %32\n\tv_add_f32 %14, %14, %32\n\t"
            "v_add_f32 %15, %15, %32\n\tv_add_f32 %16, %16, %32\n\tv_add_f32 %17, %17, %32\n\t"
            "v_add_f32 %18, %18, %32\n\tv_add_f32 %19, %19, %32\n\tv_add_f32 %20, %20, %32\n\t"
            "v_add_f32 %21, %21, %32\n\tv_add_f32 %22, %22, %32\n\tv_add_f32 %23, %23, %32\n\t"
            "v_add_f32 %24, %24, %32\n\tv_add_f32 %25, %25, %32\n\tv_add_f32 %26, %26, %32\n\t"
            "v_add_f32 %27, %27, %32\n\tv_add_f32 %28, %28, %32\n\tv_add_f32 %29, %29, %32\n\t"
            "v_add_f32 %30, %30, %32\n\tv_add_f32 %31, %31, %32"
            : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]), "+v"(a[7]),
              "+v"(a[8]), "+v"(a[9]), "+v"(a[10]), "+v"(a[11]), "+v"(a[12]), "+v"(a[13]), "+v"(a[14]), "+v"(a[15]),
              "+v"(a[16]), "+v"(a[17]), "+v"(a[18]), "+v"(a[19]), "+v"(a[20]), "+v"(a[21]), "+v"(a[22]),
              "+v"(a[23]), "+v"(a[24]), "+v"(a[25]), "+v"(a[26]), "+v"(a[27]), "+v"(a[28]), "+v"(a[29]),
              "+v"(a[30]), "+v"(a[31])
            : "v"(b));
    }
    float t = 0.f;
#pragma unroll
    for (int j = 0; j < 32; ++j) t += a[j];
    if (t == 12345.f) out[0] = t;
}
constexpr int kAddValu = 32;

// One instruction class at a time (16 independent chains an iteration), to
// see what each costs: CLS 0 v_dot2_f32_f16 accumulating, 1 v_max_f32 with a
// DPP wave shift (the shifted operand is never written in the loop, so no
// DPP hazard arises), 2 v_max3_f32.
template <int CLS>
__global__ __launch_bounds__(kProbeThreads) void k_probe_valu_class(int iters, float* out)
{
    float acc[16];
    uint32_t src[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        acc[j] = (float)j * 1e-3f;
        src[j] = ((uint32_t)(threadIdx.x + 7 * j) & 0x3ff) | 0x38003800u;
    }
    const uint32_t rh = 0x39a839a8u;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 16; j += 4) {
            if constexpr (CLS == 0)
                asm volatile(
                    "v_dot2_f32_f16 %0, %4, %5, %0\n\tv_dot2_f32_f16 %1, %4, %6, %1\n\t"
                    "v_dot2_f32_f16 %2, %4, %7, %2\n\tv_dot2_f32_f16 %3, %4, %8, %3"
                    : "+v"(acc[j]), "+v"(acc[j + 1]), "+v"(acc[j + 2]), "+v"(acc[j + 3])
                    : "s"(rh), "v"(src[j]), "v"(src[j + 1]), "v"(src[j + 2]), "v"(src[j + 3]));
            else if constexpr (CLS == 1)
                asm volatile(
                    "v_max_f32_dpp %0, %4, %0 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                    "v_max_f32_dpp %1, %5, %1 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                    "v_max_f32_dpp %2, %6, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
                    "v_max_f32_dpp %3, %7, %3 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                    : "+v"(acc[j]), "+v"(acc[j + 1]), "+v"(acc[j + 2]), "+v"(acc[j + 3])
                    : "v"(src[j]), "v"(src[j + 1]), "v"(src[j + 2]), "v"(src[j + 3]));
            else
                asm volatile(
                    "v_max3_f32 %0, %0, %4, %5\n\tv_max3_f32 %1, %1, %5, %6\n\t"
                    "v_max3_f32 %2, %2, %6, %7\n\tv_max3_f32 %3, %3, %7, %4"
                    : "+v"(acc[j]), "+v"(acc[j + 1]), "+v"(acc[j + 2]), "+v"(acc[j + 3])
                    : "v"(src[j]), "v"(src[j + 1]), "v"(src[j + 2]), "v"(src[j + 3]));
        }
    }
    float t = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) t += acc[j];
    if (t == 12345.f) out[0] = t;
}
constexpr int kClassValu = 16;

// LDS reads of the search kernel's pattern: a 64-word-wide tile, each lane
// reading its column in 10 consecutive rows from a wave-uniform offset that
// moves every iteration.
constexpr int kProbeLdsWords = 64 * 96;  // 24 KB tile
__global__ __launch_bounds__(kProbeThreads) void k_probe_lds(int iters, float* out)
{
    __shared__ float tile[kProbeLdsWords];
    for (int i = threadIdx.x; i < kProbeLdsWords; i += blockDim.x) tile[i] = (float)(i & 1023);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    float acc = 0.f;
    int off = (int)(threadIdx.x >> 6) * 3;
    for (int it = 0; it < iters; ++it) {
        // wave-uniform offset inside the tile (rows 0..85, columns 0..0)
        off = __builtin_amdgcn_readfirstlane((off * 5 + 17) % 86);
        const float* p = tile + off * 64 + lane;
        float s = 0.f;
#pragma unroll
        for (int r = 0; r < 10; ++r) s += p[r * 64];
        acc += s;
    }
    if (acc == -1.f) out[0] = acc;
}
constexpr int kLdsBytesPerIter = 10 * 4;  // per lane

// HBM stream: dst[i] = src[i] over n 16-byte words, grid-stride.
__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                              long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t launch_probe(int kind, int iters, void* buf, long long buf_bytes, hipStream_t s, double* work)
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    // eight waves per SIMD: four SIMDs a CU, four waves a workgroup
    const int blocks = cus * 8;
    const double waves = (double)blocks * (kProbeThreads / 64);
    float* out = reinterpret_cast<float*>(buf);
    switch (kind) {
        case 0:
            hipLaunchKernelGGL(k_probe_valu_mix, dim3(blocks), dim3(kProbeThreads), 0, s, iters, out);
            *work = waves * iters * kMixValu;  // wave-level VALU instructions
            break;
        case 1:
            hipLaunchKernelGGL(k_probe_valu_add, dim3(blocks), dim3(kProbeThreads), 0, s, iters, out);
            *work = waves * iters * kAddValu;
            break;
        case 2:
            hipLaunchKernelGGL(k_probe_lds, dim3(blocks), dim3(kProbeThreads), 0, s, iters, out);
            *work = waves * 64.0 * iters * kLdsBytesPerIter;  // bytes read from LDS
            break;
        case 4:
        case 5:
        case 6:
            if (kind == 4) hipLaunchKernelGGL(k_probe_valu_class<0>, dim3(blocks), dim3(kProbeThreads), 0, s, iters, out);
            if (kind == 5) hipLaunchKernelGGL(k_probe_valu_class<1>, dim3(blocks), dim3(kProbeThreads), 0, s, iters, out);
            if (kind == 6) hipLaunchKernelGGL(k_probe_valu_class<2>, dim3(blocks), dim3(kProbeThreads), 0, s, iters, out);
            *work = waves * iters * kClassValu;
            break;
        case 3: {
            const long long n = buf_bytes / 2 / 16;
            const float4* src = reinterpret_cast<const float4*>(buf);
            float4* dst = reinterpret_cast<float4*>(reinterpret_cast<char*>(buf) + n * 16);
            hipLaunchKernelGGL(k_probe_copy, dim3(cus * 16), dim3(kProbeThreads), 0, s, src, dst, n);
            *work = 2.0 * (double)n * 16;  // bytes read plus bytes written
            break;
        }
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tmk
