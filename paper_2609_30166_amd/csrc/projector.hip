// Ray-driven forward projector and its exact-transpose backprojector (gfx950).
//
// One workgroup owns a 16x16 detector tile of one projection; each lane owns
// one pixel ray.  The four wave64s of a workgroup take 8x8 quadrants so that
// the 64 rays of a wave sample a compact patch of the volume at every step.
// Workgroup ids are swizzled so that each XCD walks a contiguous run of
// (tile, projection) pairs: consecutive projections of one tile revisit almost
// the same voxels, which then stay in that XCD's L2.
//
// Per ray (Sec. 4.1, projection operator; Sec. 2.2 geometry):
//   FP64: direction M^-1 (u, v, 1), slab clip to the voxel-centre hull,
//         n = ceil(L / step), h = L / n, samples t_in + (i + 1/2) h, the
//         first sample and the step rounded to 64-bit fixed point;
//   integer: sample positions stepped exactly in fixed point;
//   FP32: fractions, optional warp c' = c + tau U(c) (Sec. 3.1, 4.2.1),
//         trilinear lookups, FP32 accumulation; sub-views averaged
//         (Sec. 3.4, 4.2.2).
// The backprojector (backproject.hip) walks the same samples with the same
// arithmetic, so it is the transpose of this operator sample by sample.

#include "ray_common.h"

namespace ctrex {
namespace {

using namespace dev;

// ------------------------------------------------------- forward kernel ----
// Gather from a corner-packed copy: the eight corners of a sample are the two
// 16-byte elements of its lower corner in slices z and z + 1, holding the
// values of the pair loads of `gather` / `gather_t` in the same order.
__device__ __forceinline__ float gather_p4(const float4 *__restrict__ p4, const VolDims &d,
                                           const Corner &k) {
    const float4 a = p4[k.base];
    const float4 b = p4[k.base + d.nxy];
    return blend(k, a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w);
}

// 16-bit volumes: the four corners of a slice are one 8-byte element, two to a
// 32-bit word (low half first), widened exactly as `ld` widens them.
__device__ __forceinline__ float widen_lo(bf16_t, uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float widen_hi(bf16_t, uint32_t w) {
    return __uint_as_float(w & 0xffff0000u);
}
__device__ __forceinline__ float widen_lo(_Float16, uint32_t w) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w)));
}
__device__ __forceinline__ float widen_hi(_Float16, uint32_t w) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w >> 16)));
}

template <typename TV>
__device__ __forceinline__ float gather_p2(const uint2 *__restrict__ p2, const VolDims &d,
                                           const Corner &k) {
    const uint2 a = p2[k.base];
    const uint2 b = p2[k.base + d.nxy];
    const TV t{};
    return blend(k, widen_lo(t, a.x), widen_hi(t, a.x), widen_lo(t, a.y), widen_hi(t, a.y),
                 widen_lo(t, b.x), widen_hi(t, b.x), widen_lo(t, b.y), widen_hi(t, b.y));
}

// The packed gather for the volume's storage type: float4 elements for FP32,
// uint2 elements for 16-bit volumes.
template <typename TV>
__device__ __forceinline__ float gather_pk(const void *__restrict__ pk, const VolDims &d,
                                           const Corner &k) {
    if constexpr (sizeof(TV) == 4)
        return gather_p4(static_cast<const float4 *>(pk), d, k);
    else
        return gather_p2<TV>(static_cast<const uint2 *>(pk), d, k);
}

// Value of the sample at fixed-point position (px, py, pz): its trilinear
// lookup (0 for a warped sample outside the hull; in the ray-length mode, 1
// inside and 0 outside).  TL: gather from the y-fastest copy; PK: from the
// corner-packed copy `pk` (y-fastest when TL; element type by TV).
template <typename TV, int MODE, bool WARP, bool TL, bool PK>
__device__ __forceinline__ float sample_value(const TV *__restrict__ vol,
                                              const void *__restrict__ pk, const VolDims &d,
                                              const WarpGrid &w, float tau, long long px,
                                              long long py, long long pz) {
    int ix, iy, iz;
    Corner k;
    const bool in = sample_corner<WARP>(d, w, tau, px, py, pz, ix, iy, iz, k.fx, k.fy, k.fz);
    if (MODE == FP_RECIP_ONES) return in ? 1.0f : 0.0f;
    k.base = TL ? base_t(d, ix, iy, iz) : base_x(d, ix, iy, iz);
    const float v = PK   ? gather_pk<TV>(pk, d, k)
                    : TL ? gather_t(vol, d, k)
                         : gather(vol, d, k);
    return in ? v : 0.0f;
}

// One ray's projection value: the mean over sub-views of the step-weighted
// trilinear samples, two samples per loop iteration (independent gathers).
template <typename TV, int MODE, bool WARP, bool TL, bool PK>
__device__ __forceinline__ float march(const RayGrid &g, const WarpGrid &w,
                                       const TV *__restrict__ vol,
                                       const void *__restrict__ pk, const VolDims &d,
                                       const TileCoord &t) {
    float y = 0.0f;
    for (int s = 0; s < g.n_sub; ++s) {
        const SubView &sv = g.tab[t.p * g.n_sub + s];
        Ray r;
        if (!setup_ray(sv, static_cast<double>(t.iu), static_cast<double>(t.iv), g.nx, g.ny,
                       g.nz, g.step, r))
            continue;
        const float tau = static_cast<float>(sv.tau);
        float acc0 = 0.0f, acc1 = 0.0f;
        long long px = r.qx, py = r.qy, pz = r.qz;
        int i = 0;
        for (; i + 1 < r.n; i += 2) {
            acc0 += sample_value<TV, MODE, WARP, TL, PK>(vol, pk, d, w, tau, px, py, pz);
            acc1 += sample_value<TV, MODE, WARP, TL, PK>(vol, pk, d, w, tau, px + r.tx,
                                                         py + r.ty, pz + r.tz);
            px += 2 * r.tx;
            py += 2 * r.ty;
            pz += 2 * r.tz;
        }
        if (i < r.n) acc0 += sample_value<TV, MODE, WARP, TL, PK>(vol, pk, d, w, tau, px, py, pz);
        y = fmaf(r.h, acc0 + acc1, y);
    }
    return y / static_cast<float>(g.n_sub);
}

// ------------------------------------------------ LDS-staged tube gather ----
// Alternative gather for FP32 volumes without warp.  The 64 rays of a wave (an
// 8x8 pixel quadrant) are nearly parallel: the wave walks them in slabs of
// TUBE_S voxels along their common major axis, stages the box of voxels the
// slab's samples can touch (bounded from each ray's FP32 line with a margin of
// one voxel, clamped to the volume) in a wave-private LDS region, and every
// lane takes its own samples of the slab from it.  Positions, corners,
// trilinear weights and the two accumulators are those of `march`, so the
// value is bitwise the same; a slab whose box exceeds TUBE_CAP voxels, or a
// sub-view whose rays do not all advance the same way along one axis, gathers
// from global memory instead.
constexpr int TUBE_S = 8;
constexpr int TUBE_CAP = 2048;

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_max_step(float v) {
    const int o = __builtin_amdgcn_update_dpp(__float_as_int(-__builtin_inff()), __float_as_int(v),
                                              CTRL, ROWS, 0xf, false);
    return fmaxf(v, __int_as_float(o));
}

// Maximum over the wave (lanes without a value pass -inf).
__device__ __forceinline__ float wave_max_f(float x) {
    x = dpp_max_step<0x111, 0xf>(x);   // row_shr:1
    x = dpp_max_step<0x112, 0xf>(x);   // row_shr:2
    x = dpp_max_step<0x114, 0xf>(x);   // row_shr:4
    x = dpp_max_step<0x118, 0xf>(x);   // row_shr:8
    x = dpp_max_step<0x142, 0xa>(x);   // row_bcast:15 -> rows 1, 3
    x = dpp_max_step<0x143, 0xc>(x);   // row_bcast:31 -> rows 2, 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

template <int MODE>
__device__ float march_tube(const RayGrid &g, const float *__restrict__ vol, const VolDims &d,
                            const TileCoord &t, bool active, float *__restrict__ tube) {
    float y = 0.0f;
    const int lane = threadIdx.x & 63;
    const int n3[3] = {d.nx, d.ny, d.nz};
    for (int s = 0; s < g.n_sub; ++s) {
        const SubView &sv = g.tab[t.p * g.n_sub + s];
        Ray r;
        const bool ok = active && setup_ray(sv, static_cast<double>(t.iu),
                                            static_cast<double>(t.iv), g.nx, g.ny, g.nz, g.step, r);
        const unsigned long long okm = __ballot(ok);
        if (!okm) continue;   // uniform
        // common major axis and direction, from the first ray; every ray must
        // advance strictly the same way along it
        const int f = __builtin_ctzll(okm);
        const float sx = __shfl(r.fx, f, 64), sy = __shfl(r.fy, f, 64), sz = __shfl(r.fz, f, 64);
        const int ma = (fabsf(sx) >= fabsf(sy) && fabsf(sx) >= fabsf(sz)) ? 0
                       : (fabsf(sy) >= fabsf(sz) ? 1 : 2);
        const long long ta = ma == 0 ? r.tx : (ma == 1 ? r.ty : r.tz);
        const bool up = (ma == 0 ? sx : (ma == 1 ? sy : sz)) > 0.0f;
        const bool same = __all(!ok || (up ? ta > 0 : ta < 0));
        float acc0 = 0.0f, acc1 = 0.0f;
        long long px = r.qx, py = r.qy, pz = r.qz;
        const int n = ok ? r.n : 0;
        int i = 0;
        auto major_of = [&](long long qx, long long qy, long long qz) {
            int k;
            float fr;
            fx_split(ma == 0 ? qx : (ma == 1 ? qy : qz), k, fr);
            return k;
        };
        auto sample_at = [&](const float *src, int x0, int y0, int z0, int lx, int ly, int lz,
                             bool lds) {
            int ix, iy, iz;
            Corner k;
            sample_corner<false>(d, WarpGrid{}, 0.0f, px, py, pz, ix, iy, iz, k.fx, k.fy, k.fz);
            // a corner outside the staged box (never, if the bound holds)
            // falls back to the global gather
            lds = lds && static_cast<unsigned>(ix - x0) < static_cast<unsigned>(lx - 1) &&
                  static_cast<unsigned>(iy - y0) < static_cast<unsigned>(ly - 1) &&
                  static_cast<unsigned>(iz - z0) < static_cast<unsigned>(lz - 1);
            float v;
            if (lds) {
                const int lxy = lx * ly;
                const int b = ((iz - z0) * ly + (iy - y0)) * lx + (ix - x0);
                v = blend(k, src[b], src[b + 1], src[b + lx], src[b + lx + 1], src[b + lxy],
                          src[b + lxy + 1], src[b + lxy + lx], src[b + lxy + lx + 1]);
            } else {
                k.base = base_x(d, ix, iy, iz);
                v = gather(vol, d, k);
            }
            if (i & 1)
                acc1 += v;
            else
                acc0 += v;
            px += r.tx;
            py += r.ty;
            pz += r.tz;
            ++i;
        };
        if (!same) {
            while (i < n) sample_at(nullptr, 0, 0, 0, 2, 2, 2, false);
        } else {
            // major-axis index range of the wave's samples
            const int k_first = n > 0 ? major_of(px, py, pz) : 0;
            const long long lx_ = px + static_cast<long long>(n - 1) * r.tx,
                            ly_ = py + static_cast<long long>(n - 1) * r.ty,
                            lz_ = pz + static_cast<long long>(n - 1) * r.tz;
            const int k_last = n > 0 ? major_of(lx_, ly_, lz_) : 0;
            const float lo_all = n > 0 ? static_cast<float>(up ? k_first : k_last) : __builtin_inff();
            const float hi_all = n > 0 ? static_cast<float>(up ? k_last : k_first) : -__builtin_inff();
            const int kmin = static_cast<int>(-wave_max_f(-lo_all));
            const int kmax = static_cast<int>(wave_max_f(hi_all));
            // the ray's FP32 line: minor coordinates as functions of the major one
            const float b3[3] = {r.bx, r.by, r.bz}, f3[3] = {r.fx, r.fy, r.fz};
            const int mb = ma == 0 ? 1 : 0, mc = ma == 2 ? 1 : 2;
            const float ia = ok ? 1.0f / f3[ma] : 0.0f;
            const float nslab = static_cast<float>((kmax - kmin) / TUBE_S + 1);
            for (int j = 0; j < static_cast<int>(nslab); ++j) {
                // slab [sl, sh] of major indices, in the rays' direction
                const int sl = up ? kmin + j * TUBE_S : kmax - (j + 1) * TUBE_S + 1;
                const int sh = sl + TUBE_S - 1;
                int lo3[3], hi3[3];
                lo3[ma] = max(0, min(sl, n3[ma] - 2));
                hi3[ma] = min(n3[ma] - 1, sh + 1);
                float mlo[2], mhi[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int ax = q == 0 ? mb : mc;
                    const float slope = f3[ax] * ia;
                    const float m1 = b3[ax] + (static_cast<float>(sl) - b3[ma]) * slope;
                    const float m2 = b3[ax] + (static_cast<float>(sh + 1) - b3[ma]) * slope;
                    mlo[q] = ok ? fminf(m1, m2) : __builtin_inff();
                    mhi[q] = ok ? fmaxf(m1, m2) : -__builtin_inff();
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int ax = q == 0 ? mb : mc;
                    const float a = -wave_max_f(-mlo[q]), b = wave_max_f(mhi[q]);
                    lo3[ax] = max(0, min(n3[ax] - 1, static_cast<int>(floorf(a)) - 1));
                    hi3[ax] = max(0, min(n3[ax] - 1, static_cast<int>(floorf(b)) + 2));
                }
                const int lx = hi3[0] - lo3[0] + 1, ly = hi3[1] - lo3[1] + 1,
                          lz = hi3[2] - lo3[2] + 1;
                const int lxy = lx * ly, nbox = lxy * lz;
                const bool fits = nbox <= TUBE_CAP;   // uniform
                if (fits) {
                    for (int e = lane; e < nbox; e += 64) {
                        const int zz = e / lxy, rem = e - zz * lxy;
                        const int yy = rem / lx, xx = rem - yy * lx;
                        tube[e] = vol[((lo3[2] + zz) * d.ny + lo3[1] + yy) * d.nx + lo3[0] + xx];
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
                // this lane's samples whose major index lies in the slab
                while (i < n) {
                    const int k = major_of(px, py, pz);
                    if (k < sl || k > sh) break;
                    sample_at(tube, lo3[0], lo3[1], lo3[2], lx, ly, lz, fits);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            // samples beyond the slabs (none unless the index estimate erred)
            while (i < n) sample_at(nullptr, 0, 0, 0, 2, 2, 2, false);
        }
        if (ok) y = fmaf(r.h, acc0 + acc1, y);
    }
    return y / static_cast<float>(g.n_sub);
}

// Occupancy caps.  The rays gather from the corner-packed copies; with more
// concurrent rays than the caches hold their patches evict each other.
// Measured at 512^3 x 720 x 768^2 (results bitwise identical): FP32 866 ms at
// 5 waves per SIMD, 782 ms at 3, 876 ms at 2, 1066 ms at 8; 16-bit 823 ms at
// 8, 765 at 6, 711 at 5, 674 at 4, 689 at 3, 808 at 2.  The warped variants
// keep the default: their 111 registers already limit them to 4 waves, and
// capping them lower was slower (helical 256^3, 1200 x 4 sub-views of
// 512 x 256, 32^3 warp: 700 ms at 4, 714 at 3, 777 at 2).  The ray-length
// mode (no gathers) keeps the default too.
template <typename TV, int MODE, bool WARP>
constexpr int fp_max_waves() {
    return (WARP || MODE == FP_RECIP_ONES) ? 8 : (sizeof(TV) == 4 ? 3 : 4);
}

template <typename TV, typename TS, int MODE, bool WARP, bool TUBE = false>
__global__ __launch_bounds__(PROJ_THREADS) __attribute__((amdgpu_waves_per_eu(1, TUBE ? 8 : fp_max_waves<TV, MODE, WARP>())))
void fp_kernel(RayGrid g, WarpGrid w,
                                                          const TV *__restrict__ vol,
                                                          TS *__restrict__ out, FpExtra ex) {
    const TileCoord t = tile_coord(g);
    if (!t.valid) return;  // uniform over the block
    const VolDims d = vol_dims(g);
    const bool active = t.iu < g.n_u && t.iv < g.n_v;
    if constexpr (TUBE) {
        __shared__ float tube[PROJ_THREADS / 64][TUBE_CAP];
        const float y = march_tube<MODE>(g, reinterpret_cast<const float *>(vol), d, t, active,
                                         tube[threadIdx.x >> 6]);
        const int pix = (t.k * g.n_v + t.iv) * g.n_u + t.iu;
        if (MODE == FP_PLAIN) {
            if (active) st(out, pix, y);
        } else {
            double e2 = 0.0;
            if (active) {
                const float bval = ld(static_cast<const TS *>(ex.b), pix);
                const float res = bval - y;
                e2 = static_cast<double>(res) * static_cast<double>(res);
                if (MODE == FP_CORRECT) st(out, pix, (ex.R ? ex.R[pix] : ex.rscale) * res);
            }
            block_sum_store(e2, ex.partials + t.lidx);
        }
        return;
    }
    // projections whose rays run mainly along x read the y-fastest copy
    const TV *vt = static_cast<const TV *>(ex.vol_t);
    const double uc = static_cast<double>((t.iu & ~(TILE_U - 1)) + TILE_U / 2);
    const double vc = static_cast<double>((t.iv & ~(TILE_V - 1)) + TILE_V / 2);
    const bool xm = MODE != FP_RECIP_ONES && x_major(g.tab[t.p * g.n_sub], uc, vc);
    // corner-packed copies of the volume's storage type
    const void *pkx = sizeof(TV) == 4 ? static_cast<const void *>(ex.p4)
                                      : static_cast<const void *>(ex.p2);
    const void *pky = sizeof(TV) == 4 ? static_cast<const void *>(ex.p4t)
                                      : static_cast<const void *>(ex.p2t);
    const bool pk = MODE != FP_RECIP_ONES && pkx != nullptr;
    float y = 0.0f;
    if (active) {
        if (pk)
            y = (xm && pky) ? march<TV, MODE, WARP, true, true>(g, w, vol, pky, d, t)
                            : march<TV, MODE, WARP, false, true>(g, w, vol, pkx, d, t);
        else
            y = (xm && vt) ? march<TV, MODE, WARP, true, false>(g, w, vt, nullptr, d, t)
                           : march<TV, MODE, WARP, false, false>(g, w, vol, nullptr, d, t);
    }
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
            if (MODE == FP_CORRECT) st(out, pix, (ex.R ? ex.R[pix] : ex.rscale) * res);
        }
        block_sum_store(e2, ex.partials + t.lidx);
    }
}

// ------------------------------------------------------ sample counting ----
__global__ __launch_bounds__(PROJ_THREADS) void count_kernel(RayGrid g,
                                                             unsigned long long *count) {
    const TileCoord t = tile_coord(g);
    if (!t.valid) return;
    unsigned long long n = 0;
    if (t.iu < g.n_u && t.iv < g.n_v) {
        for (int s = 0; s < g.n_sub; ++s) {
            Ray r;
            if (setup_ray(g.tab[t.p * g.n_sub + s], static_cast<double>(t.iu),
                          static_cast<double>(t.iv), g.nx, g.ny, g.nz, g.step, r))
                n += static_cast<unsigned long long>(r.n);
        }
    }
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(count, n);
}

inline dim3 proj_grid(const RayGrid &g) {
    const int per = (g.total_blocks + N_XCD - 1) / N_XCD;
    return dim3(static_cast<unsigned>(per * N_XCD));
}

// FP32 volumes without warp may take the LDS-staged tube gather.
template <typename TV, typename TS, int M, bool W>
void fp_launch(dim3 grid, dim3 block, hipStream_t s, const RayGrid &g, const WarpGrid &w,
               const TV *v, TS *o, const FpExtra &ex) {
    if constexpr (!W && sizeof(TV) == 4) {
        if (g.tube) {
            hipLaunchKernelGGL((fp_kernel<TV, TS, M, false, true>), grid, block, 0, s, g, w, v, o,
                               ex);
            return;
        }
    }
    hipLaunchKernelGGL((fp_kernel<TV, TS, M, W>), grid, block, 0, s, g, w, v, o, ex);
}

template <typename TV, typename TS>
hipError_t fp_dispatch_mode(const RayGrid &g, const WarpGrid &w, const void *vol, void *out,
                            int mode, const FpExtra &ex, hipStream_t s) {
    const dim3 grid = proj_grid(g), block(PROJ_THREADS);
    const TV *v = static_cast<const TV *>(vol);
    TS *o = static_cast<TS *>(out);
    const bool wp = w.U != nullptr;
#define CTREX_FP(M, W) fp_launch<TV, TS, M, W>(grid, block, s, g, w, v, o, ex)
    if (mode == FP_PLAIN) {
        if (wp) CTREX_FP(FP_PLAIN, true); else CTREX_FP(FP_PLAIN, false);
    } else if (mode == FP_CORRECT) {
        if (wp) CTREX_FP(FP_CORRECT, true); else CTREX_FP(FP_CORRECT, false);
    } else if (mode == FP_RESIDUAL) {
        if (wp) CTREX_FP(FP_RESIDUAL, true); else CTREX_FP(FP_RESIDUAL, false);
    } else {
        return hipErrorInvalidValue;
    }
#undef CTREX_FP
    return hipGetLastError();
}

template <typename TV>
hipError_t fp_dispatch_out(const RayGrid &g, const WarpGrid &w, const void *vol, void *out,
                           int out_dtype, int mode, const FpExtra &ex, hipStream_t s) {
    switch (out_dtype) {
        case F32: return fp_dispatch_mode<TV, float>(g, w, vol, out, mode, ex, s);
        case BF16: return fp_dispatch_mode<TV, bf16_t>(g, w, vol, out, mode, ex, s);
        case F16: return fp_dispatch_mode<TV, _Float16>(g, w, vol, out, mode, ex, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_forward(const RayGrid &g, const WarpGrid &w, const void *vol, int vol_dtype,
                          void *out, int out_dtype, int mode, const FpExtra &ex,
                          hipStream_t stream) {
    if (g.total_blocks <= 0) return hipSuccess;
    if (mode == FP_RECIP_ONES) {
        const dim3 grid = proj_grid(g), block(PROJ_THREADS);
        float *o = static_cast<float *>(out);
        if (w.U)
            hipLaunchKernelGGL((fp_kernel<float, float, FP_RECIP_ONES, true>), grid, block, 0,
                               stream, g, w, nullptr, o, ex);
        else
            hipLaunchKernelGGL((fp_kernel<float, float, FP_RECIP_ONES, false>), grid, block, 0,
                               stream, g, w, nullptr, o, ex);
        return hipGetLastError();
    }
    switch (vol_dtype) {
        case F32: return fp_dispatch_out<float>(g, w, vol, out, out_dtype, mode, ex, stream);
        case BF16: return fp_dispatch_out<bf16_t>(g, w, vol, out, out_dtype, mode, ex, stream);
        case F16: return fp_dispatch_out<_Float16>(g, w, vol, out, out_dtype, mode, ex, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sample_count(const RayGrid &g, unsigned long long *count, hipStream_t stream) {
    if (g.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(count_kernel, proj_grid(g), dim3(PROJ_THREADS), 0, stream, g, count);
    return hipGetLastError();
}

}  // namespace ctrex
