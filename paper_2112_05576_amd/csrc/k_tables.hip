// Projected model tables: Eq. (2) (with a scale factor for the similarity
// pose) applied to every model point of one level at every angle
// theta_min + k*step of the level's grid and every scale, in FP64, stored as
// the integer position offset and the FP32 / FP16 rotated direction.
#include "tm_device.h"

namespace tmk {

namespace {

__global__ __launch_bounds__(256) void k_tables(const ModelPoint* __restrict__ pts, int n, int n_pad,
                                                 double theta_min, double step, int K, double sigma_min,
                                                 double sigma_step, TabEntry* __restrict__ tab)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;  // j * K + k
    const int k = m % K, j = m / K;
    if (i >= n_pad) return;
    TabEntry e;
    if (i < n) {
        double c, s;
        sincos_deg(level_theta(theta_min, step, k), &c, &s);
        int qx, qy;
        double rx, ry;
        project_point_s(pts[i], c, s, scale_of(sigma_min, sigma_step, j), &qx, &qy, &rx, &ry);
        e.qx = (int16_t)qx;
        e.qy = (int16_t)qy;
        e.rx = (float)rx;
        e.ry = (float)ry;
        __half2 h = __floats2half2_rn((float)rx, (float)ry);
        e.rh = *reinterpret_cast<uint32_t*>(&h);
    } else {
        // padding entries vote exactly 0 wherever they land
        e.qx = 0;
        e.qy = 0;
        e.rx = 0.0f;
        e.ry = 0.0f;
        e.rh = 0u;
    }
    tab[(size_t)m * n_pad + i] = e;
}

// FP64 unit direction of every model point, stored once per model level so
// that the refinement, which projects each point at 3 angles for every
// candidate, does not form the square root and the divisions again.
__global__ __launch_bounds__(256) void k_unit_dirs(const ModelPoint* __restrict__ pts, int n, double2* __restrict__ dir)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double dx, dy;
    unit_dir(pts[i], &dx, &dy);
    dir[i] = make_double2(dx, dy);
}

__global__ __launch_bounds__(256) void k_table_export(const TabEntry* __restrict__ tab, int n, int n_pad, int K,
                                                       int32_t* __restrict__ q, float* __restrict__ r)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * K) return;
    const int k = (int)(idx / n), i = (int)(idx % n);
    const TabEntry e = tab[(size_t)k * n_pad + i];
    q[2 * idx] = e.qx;
    q[2 * idx + 1] = e.qy;
    r[2 * idx] = e.rx;
    r[2 * idx + 1] = e.ry;
}

}  // namespace

hipError_t launch_tables(const ModelPoint* pts, int n, int n_pad, double theta_min, double step, int K,
                         double sigma_min, double sigma_step, int S, TabEntry* tab, hipStream_t s)
{
    dim3 grid((n_pad + 255) / 256, K * S);
    hipLaunchKernelGGL(k_tables, grid, dim3(256), 0, s, pts, n, n_pad, theta_min, step, K, sigma_min, sigma_step,
                       tab);
    return hipGetLastError();
}

hipError_t launch_unit_dirs(const ModelPoint* pts, int n, double2* dir, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unit_dirs, dim3((n + 255) / 256), dim3(256), 0, s, pts, n, dir);
    return hipGetLastError();
}

hipError_t launch_table_export(const TabEntry* tab, int n, int n_pad, int K, int32_t* q, float* r, hipStream_t s)
{
    long long tot = (long long)n * K;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_table_export, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, tab, n, n_pad, K, q, r);
    return hipGetLastError();
}

}  // namespace tmk
