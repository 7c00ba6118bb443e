// Device-side building blocks shared by the projector kernels: storage
// conversions, FP64 ray set-up, trilinear corners, the displacement warp and
// the XCD-aware block mapping.  Included by the .hip translation units only.
#pragma once

#include "ctrex_internal.h"

namespace ctrex {
namespace dev {

// ---------------------------------------------------------------- storage --
__device__ __forceinline__ float ld(const float *p, int i) { return p[i]; }
__device__ __forceinline__ float ld(const bf16_t *p, int i) {
    return __uint_as_float(static_cast<uint32_t>(p[i].bits) << 16);
}
__device__ __forceinline__ float ld(const _Float16 *p, int i) { return static_cast<float>(p[i]); }

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ void st(float *p, int i, float v) { p[i] = v; }
__device__ __forceinline__ void st(bf16_t *p, int i, float v) { p[i].bits = f32_to_bf16_rne(v); }
__device__ __forceinline__ void st(_Float16 *p, int i, float v) { p[i] = static_cast<_Float16>(v); }

// ------------------------------------------------------------- ray set-up --
// Sample i of a ray sits at b + i s (index coordinates).  The FP64 set-up
// rounds b and s once to signed 64-bit fixed point with FX = 40 fractional
// bits; every sample position is then the exact integer q + i t, reached by
// stepping (q += t) in the forward projector and by one multiply-add or by
// stepping in the backprojector, so both see the same sample bit for bit.
// Against FP64 the positions are off by at most 2^-41 (the rounding of q)
// plus i 2^-41 (that of t): under 1e-8 voxel for 4096 samples and under
// 1e-5 voxel at the 2^24-sample limit.  The integer voxel is the top word
// shifted, the fraction its next 32 bits rounded to FP32: no FP64 in the
// sample loops and no re-anchoring along the ray.
constexpr int FX = 40;

struct Ray {
    long long qx, qy, qz;   // position of sample 0, fixed point
    long long tx, ty, tz;   // step vector, fixed point
    float bx, by, bz;       // position of sample 0 in FP32 (range estimates only)
    float fx, fy, fz;       // step vector in FP32 (range estimates only)
    float h;                // sample weight (path length per sample)
    int n;                  // number of samples
};

__device__ __forceinline__ long long to_fx(double v) {
    return static_cast<long long>(rint(v * 1099511627776.0));   // v 2^FX, to nearest
}

// Integer voxel k = floor(p) and fraction f = p - k of a fixed-point
// coordinate: k from the top word, f from the top 32 fraction bits rounded to
// FP32 (so f may round up to 1.0, which the corner weights treat like any
// other fraction: weight 1 on the upper corner).
__device__ __forceinline__ void fx_split(long long p, int &k, float &f) {
    const unsigned long long u = static_cast<unsigned long long>(p);
    k = static_cast<int>(static_cast<uint32_t>(u >> 32)) >> (FX - 32);
    f = static_cast<float>(static_cast<uint32_t>(u >> (FX - 32))) * 2.3283064365386963e-10f;  // 2^-32
}

// FP64 clipping of one axis' slab.  Returns false when the ray misses.
__device__ __forceinline__ bool slab(double s, double d, double hi, double &t0, double &t1) {
    if (d == 0.0) return !(s < 0.0 || s > hi);
    const double inv = 1.0 / d;
    const double a = (0.0 - s) * inv;
    const double b = (hi - s) * inv;
    const double lo_t = a < b ? a : b;
    const double hi_t = a < b ? b : a;
    if (lo_t > t0) t0 = lo_t;
    if (hi_t < t1) t1 = hi_t;
    return true;
}

// Ray through pixel centre (u, v) of sub-view sv, in FP64: unit direction
// M^-1 (u, v, 1) / |.|, slab clip to the voxel-centre hull, n = ceil(L / step),
// h = L / n, samples at t_in + (i + 1/2) h.  Reciprocals are formed once (one
// division for the length, one per axis for the slabs); the sample count n
// is then an integer function of correctly rounded FP64 values, so it differs
// from a plain division-based evaluation only if L / step lies within an ulp
// of an integer.
__device__ __forceinline__ bool setup_ray(const SubView &sv, double u, double v, int nx, int ny,
                                          int nz, double step, Ray &r) {
    double dx = fma(sv.Mi[0], u, fma(sv.Mi[1], v, sv.Mi[2]));
    double dy = fma(sv.Mi[3], u, fma(sv.Mi[4], v, sv.Mi[5]));
    double dz = fma(sv.Mi[6], u, fma(sv.Mi[7], v, sv.Mi[8]));
    const double inv_len = 1.0 / sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
    dx *= inv_len;
    dy *= inv_len;
    dz *= inv_len;
    double t0 = -__builtin_inf(), t1 = __builtin_inf();
    if (!slab(sv.S[0], dx, static_cast<double>(nx - 1), t0, t1)) return false;
    if (!slab(sv.S[1], dy, static_cast<double>(ny - 1), t0, t1)) return false;
    if (!slab(sv.S[2], dz, static_cast<double>(nz - 1), t0, t1)) return false;
    if (!(t1 > t0)) return false;
    const double L = t1 - t0;
    const double nd = ceil(L / step);
    const double h = L / nd;
    const double tb = fma(0.5, h, t0);
    const double bx = fma(tb, dx, sv.S[0]);
    const double by = fma(tb, dy, sv.S[1]);
    const double bz = fma(tb, dz, sv.S[2]);
    const double sx = h * dx, sy = h * dy, sz = h * dz;
    r.qx = to_fx(bx);
    r.qy = to_fx(by);
    r.qz = to_fx(bz);
    r.tx = to_fx(sx);
    r.ty = to_fx(sy);
    r.tz = to_fx(sz);
    r.bx = static_cast<float>(bx);
    r.by = static_cast<float>(by);
    r.bz = static_cast<float>(bz);
    r.fx = static_cast<float>(sx);
    r.fy = static_cast<float>(sy);
    r.fz = static_cast<float>(sz);
    r.h = static_cast<float>(h);
    r.n = static_cast<int>(nd);
    return true;
}

// ------------------------------------------------------------ trilinear ----
struct VolDims {
    int nx, ny, nz;
    int nxy;
    float mx, my, mz;   // n - 1 as float (clamp bounds)
};

struct Corner {
    int base;           // linear index of the lower corner
    float fx, fy, fz;   // fractions in [0, 1]
};

// Lower corner and fraction on one axis of n >= 2 nodes for the position
// i + l (i integer, l the FP32 local offset), as for the coordinate clamped
// into [0, n - 1] with corner min(floor(c), n - 2).
__device__ __forceinline__ void axis_corner(int i, float l, int n, int &k, float &f) {
    const float fl = floorf(l);
    k = i + static_cast<int>(fl);
    f = l - fl;
    if (k < 0) {
        k = 0;
        f = 0.0f;
    }
    if (k > n - 2) {
        k = n - 2;
        f = 1.0f;
    }
}

// True when i + l lies in [0, n - 1].
__device__ __forceinline__ bool axis_inside(int i, float l, int n) {
    const float fl = floorf(l);
    const int k = i + static_cast<int>(fl);
    return k >= 0 && (k < n - 1 || (k == n - 1 && l == fl));
}

// The same for a position already split into k + f with f in [0, 1): only
// the clamps (k < 0 rounds onto the first corner with weight 0 on the next;
// k > n - 2 is the last face, weight 1 on it).
__device__ __forceinline__ void axis_clamp(int k, float f, int n, int &kc, float &fc) {
    kc = k;
    fc = f;
    if (k < 0) {
        kc = 0;
        fc = 0.0f;
    }
    if (k > n - 2) {
        kc = n - 2;
        fc = 1.0f;
    }
}

__device__ __forceinline__ int base_x(const VolDims &d, int ix, int iy, int iz) {
    return (iz * d.ny + iy) * d.nx + ix;
}

// Trilinear blend of the eight corner values (x first, then y, then z).
__device__ __forceinline__ float blend(const Corner &k, float v000, float v001, float v010,
                                       float v011, float v100, float v101, float v110,
                                       float v111) {
    const float a00 = fmaf(k.fx, v001 - v000, v000);
    const float a01 = fmaf(k.fx, v011 - v010, v010);
    const float a10 = fmaf(k.fx, v101 - v100, v100);
    const float a11 = fmaf(k.fx, v111 - v110, v110);
    const float b0 = fmaf(k.fy, a01 - a00, a00);
    const float b1 = fmaf(k.fy, a11 - a10, a10);
    return fmaf(k.fz, b1 - b0, b0);
}

template <typename TV>
__device__ __forceinline__ float gather(const TV *__restrict__ vol, const VolDims &d,
                                        const Corner &k) {
    const int b = k.base;
    return blend(k, ld(vol, b), ld(vol, b + 1), ld(vol, b + d.nx), ld(vol, b + d.nx + 1),
                 ld(vol, b + d.nxy), ld(vol, b + d.nxy + 1), ld(vol, b + d.nxy + d.nx),
                 ld(vol, b + d.nxy + d.nx + 1));
}

// FP32 volumes: each x-adjacent pair of corners is one 8-byte load (4-byte
// aligned; gfx950 global loads accept it), halving the gather instructions.
typedef float f32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

template <>
__device__ __forceinline__ float gather<float>(const float *__restrict__ vol, const VolDims &d,
                                               const Corner &k) {
    const int b = k.base;
    const f32x2_a4 p00 = *reinterpret_cast<const f32x2_a4 *>(vol + b);
    const f32x2_a4 p01 = *reinterpret_cast<const f32x2_a4 *>(vol + b + d.nx);
    const f32x2_a4 p10 = *reinterpret_cast<const f32x2_a4 *>(vol + b + d.nxy);
    const f32x2_a4 p11 = *reinterpret_cast<const f32x2_a4 *>(vol + b + d.nxy + d.nx);
    return blend(k, p00.x, p00.y, p01.x, p01.y, p10.x, p10.y, p11.x, p11.y);
}

// The same gathers from a y-fastest copy of the volume ([nz][nx][ny]), used
// for projections whose rays run mainly along x: a wave's samples then spread
// over y and z, and with y fastest its neighbouring samples share cache lines
// again.  The corner values and the blend are exactly those of `gather`.
__device__ __forceinline__ int base_t(const VolDims &d, int ix, int iy, int iz) {
    return (iz * d.nx + ix) * d.ny + iy;
}

template <typename TV>
__device__ __forceinline__ float gather_t(const TV *__restrict__ vt, const VolDims &d,
                                          const Corner &k) {
    const int b = k.base;
    return blend(k, ld(vt, b), ld(vt, b + d.ny), ld(vt, b + 1), ld(vt, b + d.ny + 1),
                 ld(vt, b + d.nxy), ld(vt, b + d.nxy + d.ny), ld(vt, b + d.nxy + 1),
                 ld(vt, b + d.nxy + d.ny + 1));
}

template <>
__device__ __forceinline__ float gather_t<float>(const float *__restrict__ vt, const VolDims &d,
                                                 const Corner &k) {
    const int b = k.base;
    const f32x2_a4 q00 = *reinterpret_cast<const f32x2_a4 *>(vt + b);               // (x, z)
    const f32x2_a4 q01 = *reinterpret_cast<const f32x2_a4 *>(vt + b + d.ny);        // (x+1, z)
    const f32x2_a4 q10 = *reinterpret_cast<const f32x2_a4 *>(vt + b + d.nxy);       // (x, z+1)
    const f32x2_a4 q11 = *reinterpret_cast<const f32x2_a4 *>(vt + b + d.nxy + d.ny);
    return blend(k, q00.x, q01.x, q00.y, q01.y, q10.x, q11.x, q10.y, q11.y);
}

// True when the central ray of the tile containing pixel (u, v) of sub-view
// `sv` runs more along x than along y (uniform over a workgroup).
__device__ __forceinline__ bool x_major(const SubView &sv, double u, double v) {
    const double dx = sv.Mi[0] * u + sv.Mi[1] * v + sv.Mi[2];
    const double dy = sv.Mi[3] * u + sv.Mi[4] * v + sv.Mi[5];
    return fabs(dx) > fabs(dy);
}

// ----------------------------------------------------------------- warp ----
// Displacement at the sample k + f (per axis: integer voxel and fraction):
// the node grid coordinate (k + f) (g - 1) / (n - 1) is formed in FP32 (it
// is at most g - 1, so its rounding is ~2^-19 of a grid cell) and U is
// interpolated trilinearly there, lookups clamped to the grid.
__device__ __forceinline__ float3 displacement(const WarpGrid &w, int kx, float fx, int ky,
                                               float fy, int kz, float fz) {
    const float gx = fmaf(fx, w.fsx, static_cast<float>(kx) * w.fsx);
    const float gy = fmaf(fy, w.fsy, static_cast<float>(ky) * w.fsy);
    const float gz = fmaf(fz, w.fsz, static_cast<float>(kz) * w.fsz);
    int ix, iy, iz;
    float ax, ay, az;
    axis_corner(0, gx, w.gx, ix, ax);
    axis_corner(0, gy, w.gy, iy, ay);
    axis_corner(0, gz, w.gz, iz, az);
    const int sy = w.gx, sz = w.gx * w.gy;
    const int b = (iz * w.gy + iy) * w.gx + ix;
    const float4 u000 = w.U[b], u001 = w.U[b + 1], u010 = w.U[b + sy], u011 = w.U[b + sy + 1];
    const float4 u100 = w.U[b + sz], u101 = w.U[b + sz + 1];
    const float4 u110 = w.U[b + sz + sy], u111 = w.U[b + sz + sy + 1];
    float3 r;
#define CTREX_LERP3(c)                                              \
    {                                                               \
        const float a00 = fmaf(ax, u001.c - u000.c, u000.c);        \
        const float a01 = fmaf(ax, u011.c - u010.c, u010.c);        \
        const float a10 = fmaf(ax, u101.c - u100.c, u100.c);        \
        const float a11 = fmaf(ax, u111.c - u110.c, u110.c);        \
        const float b0 = fmaf(ay, a01 - a00, a00);                  \
        const float b1 = fmaf(ay, a11 - a10, a10);                  \
        r.c = fmaf(az, b1 - b0, b0);                                \
    }
    CTREX_LERP3(x)
    CTREX_LERP3(y)
    CTREX_LERP3(z)
#undef CTREX_LERP3
    return r;
}

// Lower corner (ix, iy, iz) and fractions of the sample at fixed-point
// position (px, py, pz), after the pull-back warp c + tau U(c) (Sec. 3.1)
// when WARP; false if the warped sample leaves the hull.  The corner is
// always set and clamped into the grid, also for a sample outside (callers
// may form its address before discarding its value).  The forward and back
// projectors call this one function, so their corners and weights agree bit
// for bit.
template <bool WARP>
__device__ __forceinline__ bool sample_corner(const VolDims &d, const WarpGrid &w, float tau,
                                              long long px, long long py, long long pz, int &ix,
                                              int &iy, int &iz, float &fx, float &fy,
                                              float &fz) {
    int kx, ky, kz;
    float lx, ly, lz;
    fx_split(px, kx, lx);
    fx_split(py, ky, ly);
    fx_split(pz, kz, lz);
    if (WARP) {
        const float3 u = displacement(w, kx, lx, ky, ly, kz, lz);
        lx = fmaf(tau, u.x, lx);
        ly = fmaf(tau, u.y, ly);
        lz = fmaf(tau, u.z, lz);
        const bool in =
            axis_inside(kx, lx, d.nx) && axis_inside(ky, ly, d.ny) && axis_inside(kz, lz, d.nz);
        axis_corner(kx, lx, d.nx, ix, fx);
        axis_corner(ky, ly, d.ny, iy, fy);
        axis_corner(kz, lz, d.nz, iz, fz);
        return in;
    } else {
        axis_clamp(kx, lx, d.nx, ix, fx);
        axis_clamp(ky, ly, d.ny, iy, fy);
        axis_clamp(kz, lz, d.nz, iz, fz);
    }
    return true;
}

// ------------------------------------------------------------- tiling ------
struct TileCoord {
    int k;      // position in the view list
    int p;      // projection index
    int iu, iv; // pixel of this lane
    int lidx;   // logical block index
    bool valid; // logical block exists
};

// XCD-aware block -> (tile, projection) mapping.  Hardware hands workgroup b
// to XCD b mod 8; logical block L = xcd * per + b / 8 gives every XCD one
// contiguous run of L, and L enumerates projections fastest within a tile.
__device__ __forceinline__ TileCoord tile_coord(const RayGrid &g) {
    TileCoord t;
    const int per = (g.total_blocks + N_XCD - 1) / N_XCD;
    const int b = blockIdx.x;
    const int L = (b % N_XCD) * per + b / N_XCD;
    t.lidx = L;
    t.valid = L < g.total_blocks;
    const int Lc = t.valid ? L : 0;
    t.k = Lc % g.n_views;
    const int tile = Lc / g.n_views;
    const int tu = tile % g.tiles_u;
    const int tv = tile / g.tiles_u;
    t.p = g.views ? g.views[t.k] : t.k;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    t.iu = tu * TILE_U + (wave & 1) * 8 + (lane & 7);
    t.iv = tv * TILE_V + (wave >> 1) * 8 + (lane >> 3);
    return t;
}

__device__ __forceinline__ VolDims vol_dims(const RayGrid &g) {
    VolDims d;
    d.nx = g.nx;
    d.ny = g.ny;
    d.nz = g.nz;
    d.nxy = g.nx * g.ny;
    d.mx = static_cast<float>(g.nx - 1);
    d.my = static_cast<float>(g.ny - 1);
    d.mz = static_cast<float>(g.nz - 1);
    return d;
}

// Block-wide sum of one double per lane into partials[L] (deterministic order).
__device__ __forceinline__ void block_sum_store(double v, double *out) {
    __shared__ double red[PROJ_THREADS / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < PROJ_THREADS / 64; ++i) s += red[i];
        *out = s;
    }
}


}  // namespace dev
}  // namespace ctrex
