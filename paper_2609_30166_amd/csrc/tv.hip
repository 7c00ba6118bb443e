// Isotropic total variation of a volume and its gradient (the regulariser of
// the differentiable reconstruction loss ||A x - b||^2 + lambda TV(x)).
//
//   TV(x) = sum_j sqrt(|D x_j|^2 + eps^2),  D = forward differences with a zero
//   difference at the last index of each axis,
//   dTV/dx_j = -(Dx_j + Dy_j + Dz_j) / m_j + Dx_{j-ex} / m_{j-ex}
//              + Dy_{j-ey} / m_{j-ey} + Dz_{j-ez} / m_{j-ez}.
//
// One thread per voxel; the stencil reads stay in L1/L2, so both kernels are
// single HBM streams (value: one volume read; gradient: one read, one write).

#include "ctrex_internal.h"

namespace ctrex {
namespace {

constexpr int TV_THREADS = 256;

struct TvDims {
    int nx, ny, nz;
    size_t nxy, n;
};

__device__ __forceinline__ void diffs(const float *__restrict__ x, const TvDims &d, int ix, int iy,
                                      int iz, size_t j, float &dx, float &dy, float &dz) {
    const float v = x[j];
    dx = ix + 1 < d.nx ? x[j + 1] - v : 0.0f;
    dy = iy + 1 < d.ny ? x[j + d.nx] - v : 0.0f;
    dz = iz + 1 < d.nz ? x[j + d.nxy] - v : 0.0f;
}

__device__ __forceinline__ float mag(float dx, float dy, float dz, float eps2) {
    return sqrtf(fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2))));
}

__global__ __launch_bounds__(TV_THREADS) void tv_value_kernel(const float *__restrict__ x,
                                                              TvDims d, float eps2,
                                                              double *__restrict__ partials) {
    __shared__ double red[TV_THREADS / 64];
    double s = 0.0;
    const size_t stride = static_cast<size_t>(gridDim.x) * TV_THREADS;
    for (size_t j = static_cast<size_t>(blockIdx.x) * TV_THREADS + threadIdx.x; j < d.n;
         j += stride) {
        const int iz = static_cast<int>(j / d.nxy);
        const size_t r = j - static_cast<size_t>(iz) * d.nxy;
        const int iy = static_cast<int>(r / d.nx);
        const int ix = static_cast<int>(r - static_cast<size_t>(iy) * d.nx);
        float dx, dy, dz;
        diffs(x, d, ix, iy, iz, j, dx, dy, dz);
        s += static_cast<double>(mag(dx, dy, dz, eps2));
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < TV_THREADS / 64; ++i) t += red[i];
        partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(TV_THREADS) void tv_grad_kernel(const float *__restrict__ x, TvDims d,
                                                             float eps2, float weight,
                                                             float *__restrict__ g) {
    const size_t stride = static_cast<size_t>(gridDim.x) * TV_THREADS;
    for (size_t j = static_cast<size_t>(blockIdx.x) * TV_THREADS + threadIdx.x; j < d.n;
         j += stride) {
        const int iz = static_cast<int>(j / d.nxy);
        const size_t r = j - static_cast<size_t>(iz) * d.nxy;
        const int iy = static_cast<int>(r / d.nx);
        const int ix = static_cast<int>(r - static_cast<size_t>(iy) * d.nx);
        float dx, dy, dz;
        diffs(x, d, ix, iy, iz, j, dx, dy, dz);
        float acc = -(dx + dy + dz) / mag(dx, dy, dz, eps2);
        float ax, ay, az;
        if (ix > 0) {
            diffs(x, d, ix - 1, iy, iz, j - 1, ax, ay, az);
            acc += ax / mag(ax, ay, az, eps2);
        }
        if (iy > 0) {
            diffs(x, d, ix, iy - 1, iz, j - d.nx, ax, ay, az);
            acc += ay / mag(ax, ay, az, eps2);
        }
        if (iz > 0) {
            diffs(x, d, ix, iy, iz - 1, j - d.nxy, ax, ay, az);
            acc += az / mag(ax, ay, az, eps2);
        }
        g[j] = weight * acc;
    }
}

}  // namespace

int tv_blocks(size_t n) {
    size_t b = (n + TV_THREADS - 1) / TV_THREADS;
    if (b > 8192) b = 8192;
    return static_cast<int>(b < 1 ? 1 : b);
}

hipError_t launch_tv_value(const float *x, int nx, int ny, int nz, float eps, double *partials,
                           hipStream_t s) {
    TvDims d{nx, ny, nz, static_cast<size_t>(nx) * ny, static_cast<size_t>(nx) * ny * nz};
    hipLaunchKernelGGL(tv_value_kernel, dim3(tv_blocks(d.n)), dim3(TV_THREADS), 0, s, x, d,
                       eps * eps, partials);
    return hipGetLastError();
}

hipError_t launch_tv_grad(const float *x, int nx, int ny, int nz, float eps, float weight,
                          float *g, hipStream_t s) {
    TvDims d{nx, ny, nz, static_cast<size_t>(nx) * ny, static_cast<size_t>(nx) * ny * nz};
    hipLaunchKernelGGL(tv_grad_kernel, dim3(tv_blocks(d.n)), dim3(TV_THREADS), 0, s, x, d,
                       eps * eps, weight, g);
    return hipGetLastError();
}

}  // namespace ctrex
