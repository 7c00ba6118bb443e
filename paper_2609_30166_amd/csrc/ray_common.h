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
struct Ray {
    float mx, my, mz;   // chord midpoint (index coordinates)
    float hx, hy, hz;   // step vector h * d
    float h;            // sample weight (path length per sample)
    float k0;           // -(n - 1) / 2: offset of sample 0 from the midpoint
    int n;              // number of samples
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
// h = L / n and the chord midpoint.  Reciprocals are formed once (one
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
    const double tm = 0.5 * (t0 + t1);
    r.mx = static_cast<float>(fma(tm, dx, sv.S[0]));
    r.my = static_cast<float>(fma(tm, dy, sv.S[1]));
    r.mz = static_cast<float>(fma(tm, dz, sv.S[2]));
    r.hx = static_cast<float>(h * dx);
    r.hy = static_cast<float>(h * dy);
    r.hz = static_cast<float>(h * dz);
    r.h = static_cast<float>(h);
    r.n = static_cast<int>(nd);
    r.k0 = -0.5f * static_cast<float>(r.n - 1);
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

// Lower corner i0 = min(floor(c), n - 2) of c clamped into [0, n - 1].
__device__ __forceinline__ Corner corner_of(const VolDims &d, float cx, float cy, float cz) {
    cx = fminf(fmaxf(cx, 0.0f), d.mx);
    cy = fminf(fmaxf(cy, 0.0f), d.my);
    cz = fminf(fmaxf(cz, 0.0f), d.mz);
    const int ix = min(static_cast<int>(cx), d.nx - 2);
    const int iy = min(static_cast<int>(cy), d.ny - 2);
    const int iz = min(static_cast<int>(cz), d.nz - 2);
    Corner k;
    k.fx = cx - static_cast<float>(ix);
    k.fy = cy - static_cast<float>(iy);
    k.fz = cz - static_cast<float>(iz);
    k.base = (iz * d.ny + iy) * d.nx + ix;
    return k;
}

// Same corner as corner_of(), returned as indices.
__device__ __forceinline__ void corner_idx(const VolDims &d, float cx, float cy, float cz, int &ix,
                                           int &iy, int &iz, float &fx, float &fy, float &fz) {
    cx = fminf(fmaxf(cx, 0.0f), d.mx);
    cy = fminf(fmaxf(cy, 0.0f), d.my);
    cz = fminf(fmaxf(cz, 0.0f), d.mz);
    ix = min(static_cast<int>(cx), d.nx - 2);
    iy = min(static_cast<int>(cy), d.ny - 2);
    iz = min(static_cast<int>(cz), d.nz - 2);
    fx = cx - static_cast<float>(ix);
    fy = cy - static_cast<float>(iy);
    fz = cz - static_cast<float>(iz);
}

template <typename TV>
__device__ __forceinline__ float gather(const TV *__restrict__ vol, const VolDims &d,
                                        const Corner &k) {
    const int b = k.base;
    const float v000 = ld(vol, b), v001 = ld(vol, b + 1);
    const float v010 = ld(vol, b + d.nx), v011 = ld(vol, b + d.nx + 1);
    const float v100 = ld(vol, b + d.nxy), v101 = ld(vol, b + d.nxy + 1);
    const float v110 = ld(vol, b + d.nxy + d.nx), v111 = ld(vol, b + d.nxy + d.nx + 1);
    const float a00 = fmaf(k.fx, v001 - v000, v000);
    const float a01 = fmaf(k.fx, v011 - v010, v010);
    const float a10 = fmaf(k.fx, v101 - v100, v100);
    const float a11 = fmaf(k.fx, v111 - v110, v110);
    const float b0 = fmaf(k.fy, a01 - a00, a00);
    const float b1 = fmaf(k.fy, a11 - a10, a10);
    return fmaf(k.fz, b1 - b0, b0);
}

// ----------------------------------------------------------------- warp ----
// Displacement at c (trilinear over the node grid, clamped to the grid).
__device__ __forceinline__ float3 displacement(const WarpGrid &w, float cx, float cy, float cz) {
    float gx = fminf(fmaxf(cx * w.sx, 0.0f), static_cast<float>(w.gx - 1));
    float gy = fminf(fmaxf(cy * w.sy, 0.0f), static_cast<float>(w.gy - 1));
    float gz = fminf(fmaxf(cz * w.sz, 0.0f), static_cast<float>(w.gz - 1));
    const int ix = min(static_cast<int>(gx), w.gx - 2);
    const int iy = min(static_cast<int>(gy), w.gy - 2);
    const int iz = min(static_cast<int>(gz), w.gz - 2);
    const float fx = gx - ix, fy = gy - iy, fz = gz - iz;
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

// Warp a sample; false if the warped sample leaves the hull.
__device__ __forceinline__ bool warp(const WarpGrid &w, const VolDims &d, float tau, float &cx,
                                     float &cy, float &cz) {
    const float3 u = displacement(w, cx, cy, cz);
    cx = fmaf(tau, u.x, cx);
    cy = fmaf(tau, u.y, cy);
    cz = fmaf(tau, u.z, cz);
    return !(cx < 0.0f || cx > d.mx || cy < 0.0f || cy > d.my || cz < 0.0f || cz > d.mz);
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
