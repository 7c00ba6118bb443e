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
// Sample i of a ray sits at b + i * s (index coordinates, FP64).  Positions
// are never formed in absolute FP32 (its ulp at coordinate 512 is 3e-5):
// every segment of SEG consecutive samples starts from an FP64 anchor split
// into an integer voxel and an FP32 remainder in [0, 1), and the samples of
// the segment are the anchor remainder plus j * s in FP32 (|j| < SEG), which
// keeps positions within about 1e-6 voxel.  Forward and back projection use
// the same arithmetic, so their samples agree bit for bit.
constexpr int SEG = 32;

struct Ray {
    double bx, by, bz;  // position of sample 0
    double sx, sy, sz;  // step vector h * d
    float fx, fy, fz;   // step vector in FP32
    float h;            // sample weight (path length per sample)
    int n;              // number of samples
};

struct Anchor {
    int ix, iy, iz;     // integer part of the segment's first sample
    float ax, ay, az;   // remainder in [0, 1)
};

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
    r.bx = fma(tb, dx, sv.S[0]);
    r.by = fma(tb, dy, sv.S[1]);
    r.bz = fma(tb, dz, sv.S[2]);
    r.sx = h * dx;
    r.sy = h * dy;
    r.sz = h * dz;
    r.fx = static_cast<float>(r.sx);
    r.fy = static_cast<float>(r.sy);
    r.fz = static_cast<float>(r.sz);
    r.h = static_cast<float>(h);
    r.n = static_cast<int>(nd);
    return true;
}

// Anchor of the segment whose first sample is i.
__device__ __forceinline__ Anchor anchor_at(const Ray &r, int i) {
    const double di = static_cast<double>(i);
    const double px = fma(di, r.sx, r.bx), py = fma(di, r.sy, r.by), pz = fma(di, r.sz, r.bz);
    const double fx = floor(px), fy = floor(py), fz = floor(pz);
    Anchor a;
    a.ix = static_cast<int>(fx);
    a.iy = static_cast<int>(fy);
    a.iz = static_cast<int>(fz);
    a.ax = static_cast<float>(px - fx);
    a.ay = static_cast<float>(py - fy);
    a.az = static_cast<float>(pz - fz);
    return a;
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

// Corner of the sample at local offsets (lx, ly, lz) from anchor a.
__device__ __forceinline__ void corner_idx(const VolDims &d, const Anchor &a, float lx, float ly,
                                           float lz, int &ix, int &iy, int &iz, float &fx,
                                           float &fy, float &fz) {
    axis_corner(a.ix, lx, d.nx, ix, fx);
    axis_corner(a.iy, ly, d.ny, iy, fy);
    axis_corner(a.iz, lz, d.nz, iz, fz);
}

__device__ __forceinline__ Corner corner_of(const VolDims &d, const Anchor &a, float lx, float ly,
                                            float lz) {
    int ix, iy, iz;
    Corner k;
    corner_idx(d, a, lx, ly, lz, ix, iy, iz, k.fx, k.fy, k.fz);
    k.base = (iz * d.ny + iy) * d.nx + ix;
    return k;
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
__device__ __forceinline__ Corner corner_of_t(const VolDims &d, const Anchor &a, float lx,
                                              float ly, float lz) {
    int ix, iy, iz;
    Corner k;
    corner_idx(d, a, lx, ly, lz, ix, iy, iz, k.fx, k.fy, k.fz);
    k.base = (iz * d.nx + ix) * d.ny + iy;
    return k;
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
// The displacement grid is anchored like the ray: per segment, the grid
// coordinate (b + i s) (g - 1) / (n - 1) of its first sample is split in FP64
// into an integer node and an FP32 remainder, and the samples of the segment
// add j times the FP32 grid step, so the trilinear weights of U are as exact
// as the sample positions.
struct GridAnchor {
    int ix, iy, iz;      // integer grid node of the segment's first sample
    float ax, ay, az;    // remainder in [0, 1)
    float sx, sy, sz;    // grid step per sample
};

__device__ __forceinline__ GridAnchor grid_anchor(const WarpGrid &w, double bx, double by,
                                                  double bz, double sx, double sy, double sz,
                                                  int i) {
    const double di = static_cast<double>(i);
    const double px = fma(di, sx, bx) * w.sx, py = fma(di, sy, by) * w.sy,
                 pz = fma(di, sz, bz) * w.sz;
    const double fx = floor(px), fy = floor(py), fz = floor(pz);
    GridAnchor a;
    a.ix = static_cast<int>(fx);
    a.iy = static_cast<int>(fy);
    a.iz = static_cast<int>(fz);
    a.ax = static_cast<float>(px - fx);
    a.ay = static_cast<float>(py - fy);
    a.az = static_cast<float>(pz - fz);
    a.sx = static_cast<float>(sx * w.sx);
    a.sy = static_cast<float>(sy * w.sy);
    a.sz = static_cast<float>(sz * w.sz);
    return a;
}

__device__ __forceinline__ GridAnchor grid_anchor(const WarpGrid &w, const Ray &r, int i) {
    return grid_anchor(w, r.bx, r.by, r.bz, r.sx, r.sy, r.sz, i);
}

// Displacement at local sample j of the anchored segment (trilinear over the
// node grid, lookups clamped to the grid).
__device__ __forceinline__ float3 displacement(const WarpGrid &w, const GridAnchor &ga, float j) {
    int ix, iy, iz;
    float fx, fy, fz;
    axis_corner(ga.ix, fmaf(j, ga.sx, ga.ax), w.gx, ix, fx);
    axis_corner(ga.iy, fmaf(j, ga.sy, ga.ay), w.gy, iy, fy);
    axis_corner(ga.iz, fmaf(j, ga.sz, ga.az), w.gz, iz, fz);
    const int sy = w.gx, sz = w.gx * w.gy;
    const int b = (iz * w.gy + iy) * w.gx + ix;
    const float4 u000 = w.U[b], u001 = w.U[b + 1], u010 = w.U[b + sy], u011 = w.U[b + sy + 1];
    const float4 u100 = w.U[b + sz], u101 = w.U[b + sz + 1];
    const float4 u110 = w.U[b + sz + sy], u111 = w.U[b + sz + sy + 1];
    float3 r;
#define CTREX_LERP3(c)                                              \
    {                                                               \
        const float a00 = fmaf(fx, u001.c - u000.c, u000.c);        \
        const float a01 = fmaf(fx, u011.c - u010.c, u010.c);        \
        const float a10 = fmaf(fx, u101.c - u100.c, u100.c);        \
        const float a11 = fmaf(fx, u111.c - u110.c, u110.c);        \
        const float b0 = fmaf(fy, a01 - a00, a00);                  \
        const float b1 = fmaf(fy, a11 - a10, a10);                  \
        r.c = fmaf(fz, b1 - b0, b0);                                \
    }
    CTREX_LERP3(x)
    CTREX_LERP3(y)
    CTREX_LERP3(z)
#undef CTREX_LERP3
    return r;
}

// Pull-back warp of local sample j (Sec. 3.1): l += tau U(sample); false if
// the warped sample leaves the hull.
__device__ __forceinline__ bool warp(const WarpGrid &w, const VolDims &d, float tau,
                                     const Anchor &a, const GridAnchor &ga, float j, float &lx,
                                     float &ly, float &lz) {
    const float3 u = displacement(w, ga, j);
    lx = fmaf(tau, u.x, lx);
    ly = fmaf(tau, u.y, ly);
    lz = fmaf(tau, u.z, lz);
    return axis_inside(a.ix, lx, d.nx) && axis_inside(a.iy, ly, d.ny) &&
           axis_inside(a.iz, lz, d.nz);
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
