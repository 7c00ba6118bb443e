// Forward projector on the aligned cylindrical domain (Sec. 3.5; the
// projector's geometry-level modification, Sec. 4.2.1).
//
// The volume is a polar grid [n_z][n_phi][n_r] about the z axis of a cylinder
// frame that a rigid pose maps the V frame to.  The host hands the kernel one
// table entry per (projection, sub-view) already in the cylinder frame: the
// source S_c and R_p M^-1, so a pixel ray's direction is R_p M^-1 (u, v, 1)
// normalised.  Per ray, in FP64: clip to the hull r <= R_h, |z| <= H (the
// infinite cylinder's quadratic and the z slab), n = ceil(L / step),
// h = L / n, sample t_i = t_in + (i + 1/2) h, position S_c + t_i d_c.  Per
// sample, in FP32: r = |(x, y)|, phi = atan2(y, x), continuous indices
// a = r / dr - 1/2 (clamped to [0, n_r - 1]: the core takes ring 0's values),
// b = phi n_phi / (2 pi) (periodic), c = z / dz + (n_z - 1) / 2, trilinear
// lookup (radial neighbours are one 8-byte load for FP32 volumes).  Sub-views
// are averaged.  Positions are FP64 until the polar map, so their error is
// the FP32 rounding of r and phi (about 1e-7 of the hull radius).
//
// The grid of workgroups and the FP_* epilogues (plain, 1/(A 1), correction
// with residual partials) are those of the Cartesian projector.

#include "ray_common.h"

namespace ctrex {
namespace {

using namespace dev;

constexpr double kTwoPi = 6.283185307179586476925287;

// Line S + t d (cylinder frame, |d| = 1) against the hull.  False if it misses.
__device__ __forceinline__ bool cyl_clip(const SubView &sv, const double d[3], const CylGrid &c,
                                         double &t0, double &t1) {
    double lo = -__builtin_inf(), hi = __builtin_inf();
    const double A = fma(d[0], d[0], d[1] * d[1]);
    const double B = fma(sv.S[0], d[0], sv.S[1] * d[1]);
    const double C = fma(sv.S[0], sv.S[0], sv.S[1] * sv.S[1]) - c.rh2;
    if (A == 0.0) {
        if (C > 0.0) return false;
    } else {
        const double disc = fma(B, B, -A * C);
        if (disc < 0.0) return false;
        const double sq = sqrt(disc);
        const double ia = 1.0 / A;
        lo = (-B - sq) * ia;
        hi = (-B + sq) * ia;
    }
    if (d[2] == 0.0) {
        if (fabs(sv.S[2]) > c.hz) return false;
    } else {
        const double iz = 1.0 / d[2];
        const double za = (-c.hz - sv.S[2]) * iz, zb = (c.hz - sv.S[2]) * iz;
        lo = fmax(lo, fmin(za, zb));
        hi = fmin(hi, fmax(za, zb));
    }
    t0 = lo;
    t1 = hi;
    return hi > lo;
}

// Unit direction of the ray through pixel (u, v) of sub-view sv (cylinder frame).
__device__ __forceinline__ void cyl_dir(const SubView &sv, double u, double v, double d[3]) {
    d[0] = fma(sv.Mi[0], u, fma(sv.Mi[1], v, sv.Mi[2]));
    d[1] = fma(sv.Mi[3], u, fma(sv.Mi[4], v, sv.Mi[5]));
    d[2] = fma(sv.Mi[6], u, fma(sv.Mi[7], v, sv.Mi[8]));
    const double il = 1.0 / sqrt(fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2])));
    d[0] *= il;
    d[1] *= il;
    d[2] *= il;
}

__device__ __forceinline__ int cyl_steps(double L, double step) {
    const int n = static_cast<int>(ceil(L / step));
    return n < 1 ? 1 : n;
}

// Two radially adjacent nodes (a0, a0 + 1) of one (slice, angle) row.
template <typename TV>
__device__ __forceinline__ float2 radial_pair(const TV *__restrict__ vol, int off) {
    return make_float2(ld(vol, off), ld(vol, off + 1));
}
typedef float f32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));
template <>
__device__ __forceinline__ float2 radial_pair<float>(const float *__restrict__ vol, int off) {
    const f32x2_a4 p = *reinterpret_cast<const f32x2_a4 *>(vol + off);
    return make_float2(p.x, p.y);
}

template <typename TV>
__device__ __forceinline__ float cyl_sample(const TV *__restrict__ vol, const CylGrid &c, float x,
                                            float y, float z) {
    const float r = sqrtf(fmaf(x, x, y * y));
    float a = fmaf(r, c.inv_dr, -0.5f);
    a = fminf(fmaxf(a, 0.0f), static_cast<float>(c.nr - 1));
    float b = atan2f(y, x) * c.phi_scale;
    if (b < 0.0f) b += static_cast<float>(c.nphi);
    float zz = fmaf(z, c.inv_dz, c.half_z);
    zz = fminf(fmaxf(zz, 0.0f), static_cast<float>(c.nz - 1));
    const int a0 = min(static_cast<int>(a), c.nr - 2);
    const int k0 = min(static_cast<int>(zz), c.nz - 2);
    const float fb_floor = floorf(b);
    int j0 = static_cast<int>(fb_floor);
    if (j0 >= c.nphi) j0 -= c.nphi;
    const int j1 = j0 + 1 == c.nphi ? 0 : j0 + 1;
    const float fa = a - static_cast<float>(a0), fz = zz - static_cast<float>(k0),
                fb = b - fb_floor;
    const int plane = c.nphi * c.nr;
    const int base = k0 * plane + a0;
    const float2 p00 = radial_pair(vol, base + j0 * c.nr);
    const float2 p01 = radial_pair(vol, base + j1 * c.nr);
    const float2 p10 = radial_pair(vol, base + plane + j0 * c.nr);
    const float2 p11 = radial_pair(vol, base + plane + j1 * c.nr);
    const float q00 = fmaf(fa, p00.y - p00.x, p00.x), q01 = fmaf(fa, p01.y - p01.x, p01.x);
    const float q10 = fmaf(fa, p10.y - p10.x, p10.x), q11 = fmaf(fa, p11.y - p11.x, p11.x);
    const float s0 = fmaf(fb, q01 - q00, q00), s1 = fmaf(fb, q11 - q10, q10);
    return fmaf(fz, s1 - s0, s0);
}

// The same lookup from the corner-packed copy: the four (ring, angle) corners
// of slices k0 and k0 + 1 are one 16-byte element each, in the order of the
// radial pairs above.
__device__ __forceinline__ float cyl_sample_p4(const float4 *__restrict__ p4, const CylGrid &c,
                                               float x, float y, float z) {
    const float r = sqrtf(fmaf(x, x, y * y));
    float a = fmaf(r, c.inv_dr, -0.5f);
    a = fminf(fmaxf(a, 0.0f), static_cast<float>(c.nr - 1));
    float b = atan2f(y, x) * c.phi_scale;
    if (b < 0.0f) b += static_cast<float>(c.nphi);
    float zz = fmaf(z, c.inv_dz, c.half_z);
    zz = fminf(fmaxf(zz, 0.0f), static_cast<float>(c.nz - 1));
    const int a0 = min(static_cast<int>(a), c.nr - 2);
    const int k0 = min(static_cast<int>(zz), c.nz - 2);
    const float fb_floor = floorf(b);
    int j0 = static_cast<int>(fb_floor);
    if (j0 >= c.nphi) j0 -= c.nphi;
    const float fa = a - static_cast<float>(a0), fz = zz - static_cast<float>(k0),
                fb = b - fb_floor;
    const int plane = c.nphi * c.nr;
    const int base = k0 * plane + j0 * c.nr + a0;
    const float4 e0 = p4[base], e1 = p4[base + plane];
    const float q00 = fmaf(fa, e0.y - e0.x, e0.x), q01 = fmaf(fa, e0.w - e0.z, e0.z);
    const float q10 = fmaf(fa, e1.y - e1.x, e1.x), q11 = fmaf(fa, e1.w - e1.z, e1.z);
    const float s0 = fmaf(fb, q01 - q00, q00), s1 = fmaf(fb, q11 - q10, q10);
    return fmaf(fz, s1 - s0, s0);
}

template <typename TV, bool PK>
__device__ __forceinline__ float cyl_lookup(const TV *__restrict__ vol,
                                            const float4 *__restrict__ p4, const CylGrid &c,
                                            float x, float y, float z) {
    return PK ? cyl_sample_p4(p4, c, x, y, z) : cyl_sample(vol, c, x, y, z);
}

template <typename TV, int MODE, bool PK>
__device__ __forceinline__ float cyl_march(const RayGrid &g, const CylGrid &c,
                                           const TV *__restrict__ vol,
                                           const float4 *__restrict__ p4, const TileCoord &t) {
    float y = 0.0f;
    for (int s = 0; s < g.n_sub; ++s) {
        const SubView &sv = g.tab[t.p * g.n_sub + s];
        double d[3], t0, t1;
        cyl_dir(sv, static_cast<double>(t.iu), static_cast<double>(t.iv), d);
        if (!cyl_clip(sv, d, c, t0, t1)) continue;
        const double L = t1 - t0;
        const int n = cyl_steps(L, g.step);
        const double h = L / n;
        if (MODE == FP_RECIP_ONES) {
            y += static_cast<float>(L);   // n samples of weight h
            continue;
        }
        // four independent samples per iteration keep several lookups in flight
        float acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f, acc3 = 0.0f;
        int i = 0;
        for (; i + 3 < n; i += 4) {
            float xs[4], ys[4], zs[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double tt = fma(i + q + 0.5, h, t0);
                xs[q] = static_cast<float>(fma(tt, d[0], sv.S[0]));
                ys[q] = static_cast<float>(fma(tt, d[1], sv.S[1]));
                zs[q] = static_cast<float>(fma(tt, d[2], sv.S[2]));
            }
            acc0 += cyl_lookup<TV, PK>(vol, p4, c, xs[0], ys[0], zs[0]);
            acc1 += cyl_lookup<TV, PK>(vol, p4, c, xs[1], ys[1], zs[1]);
            acc2 += cyl_lookup<TV, PK>(vol, p4, c, xs[2], ys[2], zs[2]);
            acc3 += cyl_lookup<TV, PK>(vol, p4, c, xs[3], ys[3], zs[3]);
        }
        for (; i < n; ++i) {
            const double tt = fma(i + 0.5, h, t0);
            acc0 += cyl_lookup<TV, PK>(vol, p4, c, static_cast<float>(fma(tt, d[0], sv.S[0])),
                                       static_cast<float>(fma(tt, d[1], sv.S[1])),
                                       static_cast<float>(fma(tt, d[2], sv.S[2])));
        }
        y = fmaf(static_cast<float>(h), (acc0 + acc1) + (acc2 + acc3), y);
    }
    return y / static_cast<float>(g.n_sub);
}

// Occupancy cap for the FP32 (polar corner-packed) gathers, as for the
// Cartesian projector: 1104 ms at the 4 waves per SIMD its registers allow,
// 1014 ms at 3, 932 ms at 2 (256 x 1608 x 512 polar grid, 720 x 768^2,
// results bitwise identical).  16-bit volumes and the ray-length mode (no
// gathers) keep the default.
template <typename TV, int MODE>
constexpr int fp_cyl_max_waves() {
    return (sizeof(TV) == 4 && MODE != FP_RECIP_ONES) ? 2 : 8;
}

template <typename TV, typename TS, int MODE>
__global__ __launch_bounds__(PROJ_THREADS) __attribute__((amdgpu_waves_per_eu(1, fp_cyl_max_waves<TV, MODE>())))
void fp_cyl_kernel(RayGrid g, CylGrid c,
                                                              const TV *__restrict__ vol,
                                                              TS *__restrict__ out, FpExtra ex) {
    const TileCoord t = tile_coord(g);
    if (!t.valid) return;  // uniform over the block
    const bool active = t.iu < g.n_u && t.iv < g.n_v;
    float y = 0.0f;
    if (active)
        y = (MODE != FP_RECIP_ONES && ex.p4) ? cyl_march<TV, MODE, true>(g, c, vol, ex.p4, t)
                                             : cyl_march<TV, MODE, false>(g, c, vol, nullptr, t);
    const int pix = (t.k * g.n_v + t.iv) * g.n_u + t.iu;
    if (MODE == FP_PLAIN) {
        if (active) st(out, pix, y);
    } else if (MODE == FP_RECIP_ONES) {
        if (active) st(out, pix, y > 0.0f ? 1.0f / y : 0.0f);
    } else {
        double e2 = 0.0;
        if (active) {
            const float bval = ld(static_cast<const TS *>(ex.b), pix);
            const float res = bval - y;
            e2 = static_cast<double>(res) * static_cast<double>(res);
            if (MODE == FP_CORRECT) st(out, pix, ex.R[pix] * res);
        }
        block_sum_store(e2, ex.partials + t.lidx);
    }
}

__global__ __launch_bounds__(PROJ_THREADS) void count_cyl_kernel(RayGrid g, CylGrid c,
                                                                 unsigned long long *count) {
    const TileCoord t = tile_coord(g);
    if (!t.valid) return;
    unsigned long long n = 0;
    if (t.iu < g.n_u && t.iv < g.n_v) {
        for (int s = 0; s < g.n_sub; ++s) {
            const SubView &sv = g.tab[t.p * g.n_sub + s];
            double d[3], t0, t1;
            cyl_dir(sv, static_cast<double>(t.iu), static_cast<double>(t.iv), d);
            if (cyl_clip(sv, d, c, t0, t1))
                n += static_cast<unsigned long long>(cyl_steps(t1 - t0, g.step));
        }
    }
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(count, n);
}

inline dim3 cyl_grid(const RayGrid &g) {
    const int per = (g.total_blocks + N_XCD - 1) / N_XCD;
    return dim3(static_cast<unsigned>(per * N_XCD));
}

template <typename TV, typename TS>
hipError_t fp_cyl_mode(const RayGrid &g, const CylGrid &c, const void *vol, void *out, int mode,
                       const FpExtra &ex, hipStream_t s) {
    const dim3 grid = cyl_grid(g), block(PROJ_THREADS);
    const TV *v = static_cast<const TV *>(vol);
    TS *o = static_cast<TS *>(out);
    switch (mode) {
    case FP_PLAIN:
        hipLaunchKernelGGL((fp_cyl_kernel<TV, TS, FP_PLAIN>), grid, block, 0, s, g, c, v, o, ex);
        break;
    case FP_CORRECT:
        hipLaunchKernelGGL((fp_cyl_kernel<TV, TS, FP_CORRECT>), grid, block, 0, s, g, c, v, o, ex);
        break;
    case FP_RESIDUAL:
        hipLaunchKernelGGL((fp_cyl_kernel<TV, TS, FP_RESIDUAL>), grid, block, 0, s, g, c, v, o,
                           ex);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TV>
hipError_t fp_cyl_out(const RayGrid &g, const CylGrid &c, const void *vol, void *out,
                      int out_dtype, int mode, const FpExtra &ex, hipStream_t s) {
    switch (out_dtype) {
    case F32: return fp_cyl_mode<TV, float>(g, c, vol, out, mode, ex, s);
    case BF16: return fp_cyl_mode<TV, bf16_t>(g, c, vol, out, mode, ex, s);
    case F16: return fp_cyl_mode<TV, _Float16>(g, c, vol, out, mode, ex, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_forward_cyl(const RayGrid &g, const CylGrid &c, const void *vol, int vol_dtype,
                              void *out, int out_dtype, int mode, const FpExtra &ex,
                              hipStream_t s) {
    if (g.total_blocks <= 0) return hipSuccess;
    if (c.nr < 2 || c.nphi < 3 || c.nz < 2) return hipErrorInvalidValue;
    if (mode == FP_RECIP_ONES) {
        hipLaunchKernelGGL((fp_cyl_kernel<float, float, FP_RECIP_ONES>), cyl_grid(g),
                           dim3(PROJ_THREADS), 0, s, g, c, nullptr, static_cast<float *>(out),
                           ex);
        return hipGetLastError();
    }
    switch (vol_dtype) {
    case F32: return fp_cyl_out<float>(g, c, vol, out, out_dtype, mode, ex, s);
    case BF16: return fp_cyl_out<bf16_t>(g, c, vol, out, out_dtype, mode, ex, s);
    case F16: return fp_cyl_out<_Float16>(g, c, vol, out, out_dtype, mode, ex, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sample_count_cyl(const RayGrid &g, const CylGrid &c, unsigned long long *count,
                                   hipStream_t s) {
    if (g.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(count_cyl_kernel, cyl_grid(g), dim3(PROJ_THREADS), 0, s, g, c, count);
    return hipGetLastError();
}

CylGrid make_cyl_grid(int nr, int nphi, int nz, double dr, double dz) {
    CylGrid c;
    c.nr = nr;
    c.nphi = nphi;
    c.nz = nz;
    c.inv_dr = static_cast<float>(1.0 / dr);
    c.inv_dz = static_cast<float>(1.0 / dz);
    c.half_z = static_cast<float>(0.5 * (nz - 1));
    c.phi_scale = static_cast<float>(nphi / kTwoPi);
    const double rh = (nr - 0.5) * dr;
    c.rh2 = rh * rh;
    c.hz = 0.5 * (nz - 1) * dz;
    return c;
}

}  // namespace ctrex
