// The paper's voxel-driven backprojector (Sec. 4.1, backprojection operator):
// every voxel centre is projected through each selected view matrix onto its
// detector image and the image is sampled bilinearly there (pixel centres at
// integer (u, v), zero beyond the border), sub-views averaged:
//     z_j (+)= (1 / n_sub) sum_{p, s} r_p(u_{p,s}(X_j), v_{p,s}(X_j)).
// It is not the transpose of the ray-driven projector; SIRT pairs it with
// C = 1 / (B 1).
//
// Gather form: one thread owns a column of KZ voxels along z and keeps their
// sums in FP64 registers over all views, then writes each voxel once, so the
// result is deterministic and needs no atomics.  A workgroup is a 16 x 16
// (x, y) patch of such columns; all its threads walk the views in the same
// order, so one view's detector footprint of the patch stays in L1 while it
// is read.  The view matrix and the view index are wave-uniform (scalar
// loads).
//
// Projection arithmetic: per (thread, view) the column's top voxel is
// projected in FP64 (a, b, w) = P (X, 1).  When the depth row of P has no
// z coefficient (every circular orbit about z), w is the same for the whole
// column and u_k = u_0 + k P[0][2] / w: the integer parts of u_0 and v_0 are
// taken in FP64 and the remainders plus k du in FP32 (|k du| < KZ pixels,
// so positions stay within about 1e-6 pixel).  Otherwise, or when the
// column's numbers are huge, each voxel is projected in FP64 on its own.
// The cost is bound by VALU issue: ~45 instructions per (voxel, view) for
// the position, the border handling, two 8-byte row loads (FP32 images) and
// the blend.

#include "ray_common.h"

namespace ctrex {
namespace {

constexpr int VB_TX = 16;
constexpr int VB_TY = 16;
constexpr int VB_THREADS = VB_TX * VB_TY;
constexpr int KZ = 8;

typedef float f32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

// Detector columns (c, c + 1) at element `off` of an image.  The byte offset
// is formed in 32 bits (images hold fewer than 2^30 pixels) and added to the
// wave-uniform image base, so the loads take the scalar-base form.
template <typename TS>
__device__ __forceinline__ const TS *at(const TS *img, unsigned off) {
    return reinterpret_cast<const TS *>(reinterpret_cast<const char *>(img) +
                                        off * static_cast<unsigned>(sizeof(TS)));
}
template <typename TS>
__device__ __forceinline__ float2 row_pair(const TS *__restrict__ img, unsigned off) {
    const TS *q = at(img, off);
    return make_float2(dev::ld(q, 0), dev::ld(q, 1));
}
template <>
__device__ __forceinline__ float2 row_pair<float>(const float *__restrict__ img, unsigned off) {
    const f32x2_a4 p = *reinterpret_cast<const f32x2_a4 *>(at(img, off));
    return make_float2(p.x, p.y);
}

// Bilinear sample of a detector image at (iu + fu, iv + fv) with zero
// outside, for iu in [-1, nu - 1] and iv in [-1, nv - 1] (nu, nv >= 2).  The
// loads stay inside the image for any (iu, iv): the column pair starts at
// c = clamp(iu, 0, nu - 2) and both rows are clamped to [0, nv - 1]; the
// weights (ea, eb) of the pair's two columns are those of columns iu and
// iu + 1 moved to where they sit in the pair (0 for a column outside).
// ONES: the sum of the in-image weights (no loads).
template <typename TS, bool ONES>
__device__ __forceinline__ float bilinear(const TS *__restrict__ img, int nu, int nv, int iu,
                                          int iv, float fu, float fv) {
    const float wt = iv >= 0 ? 1.0f - fv : 0.0f;
    const float wb = iv < nv - 1 ? fv : 0.0f;
    // iu == -1: pair (0, 1) holds column iu + 1 first; iu == nu - 1: pair
    // (nu - 2, nu - 1) holds column iu second
    const float ea = iu < 0 ? fu : (iu == nu - 1 ? 0.0f : 1.0f - fu);
    const float eb = iu < 0 ? 0.0f : (iu == nu - 1 ? 1.0f - fu : fu);
    if (ONES) return (ea + eb) * (wt + wb);
    const unsigned c = static_cast<unsigned>(min(max(iu, 0), nu - 2));
    const unsigned r0 = static_cast<unsigned>(min(max(iv, 0), nv - 1));
    const unsigned r1 = static_cast<unsigned>(min(max(iv + 1, 0), nv - 1));
    // 24-bit products (full-rate multiply; detector sides are below 2^24)
    const float2 p0 = row_pair(img, __umul24(r0, static_cast<unsigned>(nu)) + c);
    const float2 p1 = row_pair(img, __umul24(r1, static_cast<unsigned>(nu)) + c);
    return wt * fmaf(ea, p0.x, eb * p0.y) + wb * fmaf(ea, p1.x, eb * p1.y);
}

// Contribution at FP64 detector position (u, v), or 0 outside (-1, nu) x (-1, nv).
template <typename TS, bool ONES>
__device__ __forceinline__ float sample_at(const TS *__restrict__ img, int nu, int nv, double u,
                                           double v) {
    if (!(u > -1.0 && u < nu && v > -1.0 && v < nv)) return 0.0f;
    const double fu = floor(u), fv = floor(v);
    return bilinear<TS, ONES>(img, nu, nv, static_cast<int>(fu), static_cast<int>(fv),
                              static_cast<float>(u - fu), static_cast<float>(v - fv));
}

// Hardware hands workgroup b to XCD b mod 8; give every XCD one contiguous
// run of tiles (tiles enumerate z fastest, so an XCD's concurrent workgroups
// are z-neighbours whose detector footprints share rows).
__device__ __forceinline__ int xcd_tile(int b, int n_tiles) {
    const int q = n_tiles / N_XCD, rem = n_tiles % N_XCD;
    const int x = b % N_XCD;
    return x * q + min(x, rem) + b / N_XCD;
}

template <typename TS, bool ONES>
__global__ __launch_bounds__(VB_THREADS) void vbp_kernel(
    const double *__restrict__ Pm, const int *__restrict__ views, int n_views, int n_sub, int nu,
    int nv, int nx, int ny, int nz, int tiles_y, int tiles_z, const TS *__restrict__ sino,
    float *__restrict__ vol, int accumulate, VoxelGrid vg) {
    int t = xcd_tile(blockIdx.x, gridDim.x);
    const int tz = t % tiles_z;
    t /= tiles_z;
    const int ty = t % tiles_y;
    const int tx = t / tiles_y;
    const int ix = tx * VB_TX + (threadIdx.x & (VB_TX - 1));
    const int iy = ty * VB_TY + (threadIdx.x / VB_TX);
    if (ix >= nx || iy >= ny) return;  // no barriers below
    const int z0 = tz * KZ;
    const int kn = min(KZ, nz - z0);
    // the column's top voxel centre and its step along the column
    double X, Y, Z0, sz;
    if (vg.cyl) {
        // polar grid: ring ix, angle iy, slice z0
        const double r = (ix + 0.5) * vg.dr;
        const double phi = 6.283185307179586476925287 * iy / ny;
        double sn, cs;
        sincos(phi, &sn, &cs);
        X = r * cs;
        Y = r * sn;
        Z0 = (z0 - 0.5 * (nz - 1)) * vg.dz;
        sz = vg.dz;
    } else {
        X = ix - 0.5 * (nx - 1);
        Y = iy - 0.5 * (ny - 1);
        Z0 = z0 - 0.5 * (nz - 1);
        sz = 1.0;
    }
    const size_t img_px = static_cast<size_t>(nu) * nv;
    double acc[KZ];
#pragma unroll
    for (int k = 0; k < KZ; ++k) acc[k] = 0.0;

    for (int j = 0; j < n_views; ++j) {
        const int p = views ? views[j] : j;
        const TS *img = sino + (ONES ? 0 : j * img_px);
        for (int s = 0; s < n_sub; ++s) {
            const double *M = Pm + 12 * (static_cast<size_t>(p) * n_sub + s);
            const double a0 = fma(M[0], X, fma(M[1], Y, fma(M[2], Z0, M[3])));
            const double b0 = fma(M[4], X, fma(M[5], Y, fma(M[6], Z0, M[7])));
            const double w0 = fma(M[8], X, fma(M[9], Y, fma(M[10], Z0, M[11])));
            // change of (a, b, w) per voxel down the column
            const double ca = M[2] * sz, cb = M[6] * sz, cw = M[10] * sz;
            bool fast = cw == 0.0 && w0 != 0.0;
            double u0 = 0.0, v0 = 0.0, du = 0.0, dv = 0.0;
            if (fast) {
                const double r = 1.0 / w0;
                u0 = a0 * r;
                v0 = b0 * r;
                du = ca * r;
                dv = cb * r;
                fast = fabs(u0) < 16777216.0 && fabs(v0) < 16777216.0 && fabs(du) < 65536.0 &&
                       fabs(dv) < 65536.0;
            }
            if (fast) {
                // the column's u and v run linearly in k: skip it if it misses
                const double ue = fma(kn - 1.0, du, u0), ve = fma(kn - 1.0, dv, v0);
                if (!(fmax(u0, ue) > -1.0 && fmin(u0, ue) < nu && fmax(v0, ve) > -1.0 &&
                      fmin(v0, ve) < nv))
                    continue;
                const double fu0 = floor(u0), fv0 = floor(v0);
                const int iu0 = static_cast<int>(fu0), iv0 = static_cast<int>(fv0);
                const float ru = static_cast<float>(u0 - fu0), rv = static_cast<float>(v0 - fv0);
                const float duf = static_cast<float>(du), dvf = static_cast<float>(dv);
                // branch-free over the column: every voxel's loads are issued
                // (at clamped, in-image addresses) before any is consumed, and
                // voxels off the detector or past the volume are selected out
#pragma unroll
                for (int k = 0; k < KZ; ++k) {
                    const float uf = fmaf(static_cast<float>(k), duf, ru);
                    const float vf = fmaf(static_cast<float>(k), dvf, rv);
                    const int iu = iu0 + static_cast<int>(floorf(uf));
                    const int iv = iv0 + static_cast<int>(floorf(vf));
                    const bool in = k < kn &&
                                    static_cast<unsigned>(iu + 1) <= static_cast<unsigned>(nu) &&
                                    static_cast<unsigned>(iv + 1) <= static_cast<unsigned>(nv);
                    const float val = bilinear<TS, ONES>(img, nu, nv, iu, iv,
                                                         __builtin_amdgcn_fractf(uf),
                                                         __builtin_amdgcn_fractf(vf));
                    acc[k] += in ? val : 0.0f;
                }
            } else {
#pragma unroll
                for (int k = 0; k < KZ; ++k) {
                    if (k >= kn) break;
                    const double w = fma(static_cast<double>(k), cw, w0);
                    if (w == 0.0) continue;
                    const double u = fma(static_cast<double>(k), ca, a0) / w;
                    const double v = fma(static_cast<double>(k), cb, b0) / w;
                    acc[k] += sample_at<TS, ONES>(img, nu, nv, u, v);
                }
            }
        }
    }
    const double inv_sub = 1.0 / n_sub;
    const size_t col = static_cast<size_t>(iy) * nx + ix;
    const size_t plane = static_cast<size_t>(nx) * ny;
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
        if (k >= kn) break;
        float *dst = vol + (static_cast<size_t>(z0) + k) * plane + col;
        const float add = static_cast<float>(acc[k] * inv_sub);
        *dst = accumulate ? *dst + add : add;
    }
}

template <typename TS>
hipError_t launch_typed(const RayGrid &g, const double *Pm, const void *sino, float *vol,
                        int accumulate, int ones, const VoxelGrid &vg, hipStream_t s) {
    const int tiles_x = (g.nx + VB_TX - 1) / VB_TX;
    const int tiles_y = (g.ny + VB_TY - 1) / VB_TY;
    const int tiles_z = (g.nz + KZ - 1) / KZ;
    const long long n_tiles = static_cast<long long>(tiles_x) * tiles_y * tiles_z;
    if (n_tiles <= 0 || n_tiles >= (1ll << 31)) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(n_tiles)), block(VB_THREADS);
    const TS *src = static_cast<const TS *>(sino);
    if (ones)
        hipLaunchKernelGGL((vbp_kernel<TS, true>), grid, block, 0, s, Pm, g.views, g.n_views,
                           g.n_sub, g.n_u, g.n_v, g.nx, g.ny, g.nz, tiles_y, tiles_z, src, vol,
                           accumulate, vg);
    else
        hipLaunchKernelGGL((vbp_kernel<TS, false>), grid, block, 0, s, Pm, g.views, g.n_views,
                           g.n_sub, g.n_u, g.n_v, g.nx, g.ny, g.nz, tiles_y, tiles_z, src, vol,
                           accumulate, vg);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_back_voxel(const RayGrid &g, const double *Pm, const void *sino, int sino_dtype,
                             float *vol, int accumulate, int ones, const VoxelGrid &vg,
                             hipStream_t s) {
    if (g.n_views <= 0) return hipSuccess;
    if (g.n_u < 2 || g.n_v < 2 || g.n_u >= (1 << 24) || g.n_v >= (1 << 24) ||
        static_cast<long long>(g.n_u) * g.n_v >= (1ll << 30))
        return hipErrorInvalidValue;
    if (ones) return launch_typed<float>(g, Pm, nullptr, vol, accumulate, 1, vg, s);
    switch (sino_dtype) {
    case F32: return launch_typed<float>(g, Pm, sino, vol, accumulate, 0, vg, s);
    case BF16: return launch_typed<bf16_t>(g, Pm, sino, vol, accumulate, 0, vg, s);
    case F16: return launch_typed<_Float16>(g, Pm, sino, vol, accumulate, 0, vg, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ctrex
