// Voxel-space and bookkeeping kernels of the SIRT loop (Eq. 1, term 3):
// x <- x + alpha C z with z = A^T r, the reciprocal weights, the 16-bit gather
// shadows, and deterministic reductions of the per-block residual sums.
// All are single streams over HBM: 64-bit-indexed grid-stride loops with
// float4 accesses where the sizes allow.

#include "ctrex_internal.h"

namespace ctrex {
namespace {

constexpr int THREADS = 256;

__device__ __forceinline__ uint16_t bf16_rne(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ float load_as_f32(const void *p, int dt, size_t i) {
    if (dt == F32) return static_cast<const float *>(p)[i];
    if (dt == BF16)
        return __uint_as_float(static_cast<uint32_t>(static_cast<const uint16_t *>(p)[i]) << 16);
    return static_cast<float>(static_cast<const _Float16 *>(p)[i]);
}

__device__ __forceinline__ void store_from_f32(void *p, int dt, size_t i, float v) {
    if (dt == F32)
        static_cast<float *>(p)[i] = v;
    else if (dt == BF16)
        static_cast<uint16_t *>(p)[i] = bf16_rne(v);
    else
        static_cast<_Float16 *>(p)[i] = static_cast<_Float16>(v);
}

inline unsigned grid_for(size_t n) {
    size_t b = (n + THREADS - 1) / THREADS;
    if (b > 65536) b = 65536;
    if (b == 0) b = 1;
    return static_cast<unsigned>(b);
}

__global__ __launch_bounds__(THREADS) void fill_zero_kernel(uint32_t *p, size_t n_words) {
    const size_t stride = static_cast<size_t>(gridDim.x) * THREADS;
    for (size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x; i < n_words; i += stride)
        p[i] = 0u;
}

__global__ __launch_bounds__(THREADS) void fill_zero_bytes_kernel(uint8_t *p, size_t n) {
    const size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(THREADS) void recip_kernel(float *a, size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * THREADS;
    for (size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x; i < n; i += stride) {
        const float v = a[i];
        a[i] = v > 0.0f ? 1.0f / v : 0.0f;
    }
}

// x <- x + alpha C w z (w: optional voxel weights; optionally clamped at 0),
// shadow <- x.
__global__ __launch_bounds__(THREADS) void update_kernel(float *__restrict__ x,
                                                         const float *__restrict__ z,
                                                         const float *__restrict__ C,
                                                         const float *__restrict__ w, float alpha,
                                                         int nonneg, void *shadow, int sdt,
                                                         size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * THREADS;
    for (size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x; i < n; i += stride) {
        const float g = w ? alpha * C[i] * w[i] : alpha * C[i];
        float v = fmaf(g, z[i], x[i]);
        if (nonneg) v = fmaxf(v, 0.0f);
        x[i] = v;
        if (shadow) store_from_f32(shadow, sdt, i, v);
    }
}

__global__ __launch_bounds__(THREADS) void convert_kernel(const void *src, int sdt, void *dst,
                                                          int ddt, size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * THREADS;
    for (size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x; i < n; i += stride)
        store_from_f32(dst, ddt, i, load_as_f32(src, sdt, i));
}

// One block: fixed-order sum of n doubles (each thread strides, then a tree).
__global__ __launch_bounds__(1024) void sum_partials_kernel(const double *p, int n, double *out) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s += p[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Block max of |x| folded into *out with an integer max on the float bits
// (non-negative floats order like their bit patterns); NaN propagates as the
// largest pattern.
__global__ __launch_bounds__(THREADS) void max_abs_kernel(const void *x, int dt, size_t n,
                                                          unsigned *out) {
    __shared__ unsigned red[THREADS / 64];
    unsigned m = 0u;
    const size_t stride = static_cast<size_t>(gridDim.x) * THREADS;
    for (size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x; i < n; i += stride)
        m = max(m, __float_as_uint(fabsf(load_as_f32(x, dt, i))));
    for (int o = 32; o > 0; o >>= 1) m = max(m, static_cast<unsigned>(__shfl_xor(m, o, 64)));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < THREADS / 64; ++i) m = max(m, red[i]);
        atomicMax(out, m);
    }
}

__global__ __launch_bounds__(THREADS) void repack_warp_kernel(const float *U, float4 *out,
                                                              size_t n) {
    const size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x;
    if (i < n) out[i] = make_float4(U[3 * i], U[3 * i + 1], U[3 * i + 2], 0.0f);
}

// dst[z][x][y] = src[z][y][x] through 32 x 32 LDS tiles (reads and writes
// coalesced); T is the storage word (4 or 2 bytes).
template <typename T>
__global__ __launch_bounds__(256) void transpose_xy_kernel(const T *__restrict__ src,
                                                           T *__restrict__ dst, int nx, int ny) {
    __shared__ T tile[32][33];
    const size_t plane = static_cast<size_t>(blockIdx.z) * nx * ny;
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int x = x0 + tx, y = y0 + j;
        if (x < nx && y < ny) tile[j][tx] = src[plane + static_cast<size_t>(y) * nx + x];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int y = y0 + tx, x = x0 + j;
        if (x < nx && y < ny) dst[plane + static_cast<size_t>(x) * ny + y] = tile[tx][j];
    }
}

// Corner-packed copies: element (x, y, z) holds v(x, y), v(x+1, y), v(x, y+1),
// v(x+1, y+1) of slice z (indices clamped at the last row and column, whose
// elements the gathers never read).  XF: x-fastest layout, else y-fastest.
template <bool XF>
__global__ __launch_bounds__(THREADS) void pack_corners_kernel(const float *__restrict__ v,
                                                               float4 *__restrict__ out, int nx,
                                                               int ny, size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * THREADS;
    for (size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x; i < n; i += stride) {
        int x, y;
        size_t z;
        if (XF) {
            x = static_cast<int>(i % nx);
            const size_t r = i / nx;
            y = static_cast<int>(r % ny);
            z = r / ny;
        } else {
            y = static_cast<int>(i % ny);
            const size_t r = i / ny;
            x = static_cast<int>(r % nx);
            z = r / nx;
        }
        const int x1 = min(x + 1, nx - 1), y1 = min(y + 1, ny - 1);
        const float *s = v + z * nx * ny;
        out[i] = make_float4(s[static_cast<size_t>(y) * nx + x], s[static_cast<size_t>(y) * nx + x1],
                             s[static_cast<size_t>(y1) * nx + x], s[static_cast<size_t>(y1) * nx + x1]);
    }
}

template <bool XF>
__global__ __launch_bounds__(THREADS) void pack_corners16_kernel(const uint16_t *__restrict__ v,
                                                                 uint2 *__restrict__ out, int nx,
                                                                 int ny, size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * THREADS;
    for (size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x; i < n; i += stride) {
        int x, y;
        size_t z;
        if (XF) {
            x = static_cast<int>(i % nx);
            const size_t r = i / nx;
            y = static_cast<int>(r % ny);
            z = r / ny;
        } else {
            y = static_cast<int>(i % ny);
            const size_t r = i / ny;
            x = static_cast<int>(r % nx);
            z = r / nx;
        }
        const int x1 = min(x + 1, nx - 1), y1 = min(y + 1, ny - 1);
        const uint16_t *s = v + z * nx * ny;
        const uint32_t c00 = s[static_cast<size_t>(y) * nx + x],
                       c10 = s[static_cast<size_t>(y) * nx + x1];
        const uint32_t c01 = s[static_cast<size_t>(y1) * nx + x],
                       c11 = s[static_cast<size_t>(y1) * nx + x1];
        out[i] = make_uint2(c00 | (c10 << 16), c01 | (c11 << 16));
    }
}

__global__ __launch_bounds__(THREADS) void pack_polar_kernel(const float *__restrict__ v,
                                                             float4 *__restrict__ out, int nr,
                                                             int nphi, size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * THREADS;
    for (size_t i = static_cast<size_t>(blockIdx.x) * THREADS + threadIdx.x; i < n; i += stride) {
        const int a = static_cast<int>(i % nr);
        const size_t r = i / nr;
        const int j = static_cast<int>(r % nphi);
        const size_t k = r / nphi;
        const int a1 = min(a + 1, nr - 1), j1 = j + 1 == nphi ? 0 : j + 1;
        const float *s = v + k * nr * nphi;
        out[i] = make_float4(s[static_cast<size_t>(j) * nr + a], s[static_cast<size_t>(j) * nr + a1],
                             s[static_cast<size_t>(j1) * nr + a], s[static_cast<size_t>(j1) * nr + a1]);
    }
}

}  // namespace

hipError_t launch_pack_polar(const float *vol, float4 *p4, int nr, int nphi, int nz,
                             hipStream_t s) {
    const size_t n = static_cast<size_t>(nr) * nphi * nz;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(pack_polar_kernel, dim3(grid_for(n)), dim3(THREADS), 0, s, vol, p4, nr,
                       nphi, n);
    return hipGetLastError();
}

hipError_t launch_pack_corners(const float *vol, float4 *p4, float4 *p4t, int nx, int ny, int nz,
                               hipStream_t s) {
    const size_t n = static_cast<size_t>(nx) * ny * nz;
    if (n == 0) return hipSuccess;
    if (p4)
        hipLaunchKernelGGL(pack_corners_kernel<true>, dim3(grid_for(n)), dim3(THREADS), 0, s, vol,
                           p4, nx, ny, n);
    if (p4t)
        hipLaunchKernelGGL(pack_corners_kernel<false>, dim3(grid_for(n)), dim3(THREADS), 0, s,
                           vol, p4t, nx, ny, n);
    return hipGetLastError();
}

hipError_t launch_pack_corners16(const uint16_t *vol, uint2 *p2, uint2 *p2t, int nx, int ny,
                                 int nz, hipStream_t s) {
    const size_t n = static_cast<size_t>(nx) * ny * nz;
    if (n == 0) return hipSuccess;
    if (p2)
        hipLaunchKernelGGL(pack_corners16_kernel<true>, dim3(grid_for(n)), dim3(THREADS), 0, s,
                           vol, p2, nx, ny, n);
    if (p2t)
        hipLaunchKernelGGL(pack_corners16_kernel<false>, dim3(grid_for(n)), dim3(THREADS), 0, s,
                           vol, p2t, nx, ny, n);
    return hipGetLastError();
}

hipError_t launch_transpose_xy(const void *src, void *dst, int dtype, int nx, int ny, int nz,
                               hipStream_t s) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return hipSuccess;
    const dim3 grid((nx + 31) / 32, (ny + 31) / 32, nz), block(256);
    if (dtype == F32)
        hipLaunchKernelGGL(transpose_xy_kernel<uint32_t>, grid, block, 0, s,
                           static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst), nx, ny);
    else
        hipLaunchKernelGGL(transpose_xy_kernel<uint16_t>, grid, block, 0, s,
                           static_cast<const uint16_t *>(src), static_cast<uint16_t *>(dst), nx, ny);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const size_t words = bytes / 4;
    if (words) hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(words)), dim3(THREADS), 0, s,
                                  static_cast<uint32_t *>(ptr), words);
    const size_t tail = bytes - words * 4;
    if (tail)
        hipLaunchKernelGGL(fill_zero_bytes_kernel, dim3(1), dim3(THREADS), 0, s,
                           static_cast<uint8_t *>(ptr) + words * 4, tail);
    return hipGetLastError();
}

hipError_t launch_recip(float *a, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(recip_kernel, dim3(grid_for(n)), dim3(THREADS), 0, s, a, n);
    return hipGetLastError();
}

hipError_t launch_update(float *x, const float *z, const float *C, const float *w, float alpha,
                         int nonneg, void *shadow, int shadow_dtype, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(update_kernel, dim3(grid_for(n)), dim3(THREADS), 0, s, x, z, C, w, alpha,
                       nonneg, shadow, shadow_dtype, n);
    return hipGetLastError();
}

hipError_t launch_convert(const void *src, int src_dtype, void *dst, int dst_dtype, size_t n,
                          hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(convert_kernel, dim3(grid_for(n)), dim3(THREADS), 0, s, src, src_dtype,
                       dst, dst_dtype, n);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partials, int n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(1024), 0, s, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_max_abs(const void *x, int dtype, size_t n, float *out, hipStream_t s) {
    hipError_t e = launch_fill_zero(out, sizeof(float), s);
    if (e != hipSuccess || n == 0) return e;
    size_t blocks = (n + THREADS - 1) / THREADS;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(max_abs_kernel, dim3(static_cast<unsigned>(blocks)), dim3(THREADS), 0, s, x,
                       dtype, n, reinterpret_cast<unsigned *>(out));
    return hipGetLastError();
}

hipError_t launch_repack_warp(const float *U, float4 *out, size_t n_nodes, hipStream_t s) {
    if (n_nodes == 0) return hipSuccess;
    hipLaunchKernelGGL(repack_warp_kernel, dim3((n_nodes + THREADS - 1) / THREADS), dim3(THREADS),
                       0, s, U, out, n_nodes);
    return hipGetLastError();
}

}  // namespace ctrex
