// Exact-transpose backprojector with brick-resident LDS accumulation (gfx950).
//
// z += A^T r walks exactly the samples of the forward projector (same FP64
// ray set-up, same FP32 sample positions, warp and corners) and adds
// (h r / n_sub) times the eight trilinear weights of every sample to the
// volume (Sec. 4.1 backprojection operator, taken as the transpose of the
// projection operator; Sec. 3.4: a projection's residual is spread over its
// sub-views).
//
// Scattering every sample to HBM would cost eight L2 float atomics per
// sample.  Here a workgroup owns a brick of the volume (up to 32x15x16
// voxels) held in LDS for a whole chunk of projections, accumulated in FP64:
// on gfx950 the LDS FP64 atomic add sustains about twelve times the lane
// rate of the FP32 one, and the wider accumulator removes the FP32
// summation error of long sums.  For every
// (projection, sub-view) it bounds the detector pixels whose rays can reach
// the brick (the projection of the brick grown by one voxel and the warp
// bound), redoes those rays' FP64 set-up, clips their sample range to the
// grown brick, and adds with LDS float atomics the corners that fall inside
// the brick.  A sample whose corner cube straddles a brick face is visited
// by each brick it touches, and each adds only its own corners, so every
// corner is added once.  There is no global atomic and no barrier inside the
// projection loop; the brick is written out once at the end (with atomics
// only when several projection chunks share a brick).

#include "ray_common.h"

namespace ctrex {
namespace {

using namespace dev;

constexpr int BP_THREADS = 512;

struct BrickGrid {
    int bx, by, bz;       // brick size (voxels)
    int sy, sz;           // LDS row / plane strides (padded against bank conflicts)
    int nbx, nby, nbz;    // bricks per axis
    int chunks;           // projection chunks per brick
    int views_per_chunk;
    int total;            // nbx * nby * nbz * chunks
    int accumulate;       // add into vol (else overwrite; needs chunks == 1)
};

// Project the 8 corners of an index-space box through the view matrix and
// return the detector pixel range whose rays can cross the box.  When all
// corners lie on one side of the plane through the source parallel to the
// detector (w of one sign), the box's image is the hull of the corner images;
// otherwise the image is unbounded and false asks for the whole detector.
__device__ __forceinline__ bool project_box(const double *P, const double lo[3],
                                            const double hi[3], const double off[3], int n_u,
                                            int n_v, int &u0, int &u1, int &v0, int &v1) {
    double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
    bool pos = true, neg = true;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const double X = ((c & 1) ? hi[0] : lo[0]) - off[0];
        const double Y = ((c & 2) ? hi[1] : lo[1]) - off[1];
        const double Z = ((c & 4) ? hi[2] : lo[2]) - off[2];
        const double a = P[0] * X + P[1] * Y + P[2] * Z + P[3];
        const double b = P[4] * X + P[5] * Y + P[6] * Z + P[7];
        const double w = P[8] * X + P[9] * Y + P[10] * Z + P[11];
        pos = pos && w > 0.0;
        neg = neg && w < 0.0;
        const double u = a / w, v = b / w;
        umin = fmin(umin, u);
        umax = fmax(umax, u);
        vmin = fmin(vmin, v);
        vmax = fmax(vmax, v);
    }
    if (!(pos || neg)) return false;
    u0 = static_cast<int>(fmax(floor(umin) - 1.0, 0.0));
    v0 = static_cast<int>(fmax(floor(vmin) - 1.0, 0.0));
    u1 = static_cast<int>(fmin(ceil(umax) + 1.0, static_cast<double>(n_u - 1)));
    v1 = static_cast<int>(fmin(ceil(vmax) + 1.0, static_cast<double>(n_v - 1)));
    return true;
}

template <typename TS, int MODE, bool WARP>
__global__ __launch_bounds__(BP_THREADS) void bp_brick_kernel(RayGrid g, WarpGrid w,
                                                              const double *__restrict__ Pmat,
                                                              const TS *__restrict__ sino,
                                                              float *__restrict__ vol,
                                                              BrickGrid bg) {
    extern __shared__ double acc[];
    // ---- block -> (brick, projection chunk); XCD-aware so that one XCD
    // works on neighbouring bricks
    const int per = (bg.total + N_XCD - 1) / N_XCD;
    const int L = (blockIdx.x % N_XCD) * per + blockIdx.x / N_XCD;
    if (L >= bg.total) return;
    const int chunk = L % bg.chunks;
    int b = L / bg.chunks;
    const int ibx = b % bg.nbx;
    b /= bg.nbx;
    const int iby = b % bg.nby;
    const int ibz = b / bg.nby;
    const int x0 = ibx * bg.bx, y0 = iby * bg.by, z0 = ibz * bg.bz;
    const int ex = min(bg.bx, g.nx - x0), ey = min(bg.by, g.ny - y0), ez = min(bg.bz, g.nz - z0);
    const int sy = bg.sy, sz = bg.sz;
    const int nlds = sz * ez;
    for (int i = threadIdx.x; i < nlds; i += BP_THREADS) acc[i] = 0.0;
    __syncthreads();

    const VolDims d = vol_dims(g);
    const float M = static_cast<float>(w.margin);
    // samples with an (unwarped) position in [lo, hi] can touch the brick
    const float lo[3] = {x0 - 1.0f - M, y0 - 1.0f - M, z0 - 1.0f - M};
    const float hi[3] = {static_cast<float>(x0 + ex) + M, static_cast<float>(y0 + ey) + M,
                         static_cast<float>(z0 + ez) + M};
    const double lod[3] = {lo[0], lo[1], lo[2]}, hid[3] = {hi[0], hi[1], hi[2]};
    const double off[3] = {0.5 * (g.nx - 1), 0.5 * (g.ny - 1), 0.5 * (g.nz - 1)};
    const float inv_sub = 1.0f / static_cast<float>(g.n_sub);
    const int k_first = chunk * bg.views_per_chunk;
    const int k_end = min(k_first + bg.views_per_chunk, g.n_views);

    for (int k = k_first; k < k_end; ++k) {
        const int p = g.views ? g.views[k] : k;
        for (int s = 0; s < g.n_sub; ++s) {
            const int sv_idx = p * g.n_sub + s;
            const SubView &sv = g.tab[sv_idx];
            int u0 = 0, u1 = g.n_u - 1, v0 = 0, v1 = g.n_v - 1;
            if (!project_box(Pmat + 12 * static_cast<size_t>(sv_idx), lod, hid, off, g.n_u, g.n_v,
                             u0, u1, v0, v1)) {
                u0 = 0;
                u1 = g.n_u - 1;
                v0 = 0;
                v1 = g.n_v - 1;
            }
            if (u0 > u1 || v0 > v1) continue;
            // rays in 8x8 pixel blocks: one block per wave and pass, so the 64
            // samples of an LDS atomic spread over rows and columns of the brick
            const int bu = (u1 - u0 + 8) >> 3;
            const int nblk = bu * ((v1 - v0 + 8) >> 3);
            const float tau = static_cast<float>(sv.tau);
            const int lane = threadIdx.x & 63;
            for (int blk = threadIdx.x >> 6; blk < nblk; blk += BP_THREADS / 64) {
                const int iv = v0 + (blk / bu) * 8 + (lane >> 3);
                const int iu = u0 + (blk % bu) * 8 + (lane & 7);
                if (iu > u1 || iv > v1) continue;
                const float rv = (MODE == BP_ONES) ? 1.0f
                                                   : ld(sino, (k * g.n_v + iv) * g.n_u + iu);
                if (rv == 0.0f) continue;
                Ray r;
                if (!setup_ray(sv, static_cast<double>(iu), static_cast<double>(iv), g.nx, g.ny,
                               g.nz, g.step, r))
                    continue;
                // sample offsets k with mid + k h inside [lo, hi] on every axis
                float kmin = r.k0, kmax = r.k0 + static_cast<float>(r.n - 1);
                const float mv[3] = {r.mx, r.my, r.mz};
                const float hv[3] = {r.hx, r.hy, r.hz};
                bool hit = true;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (hv[a] != 0.0f) {
                        const float inv = 1.0f / hv[a];
                        const float t1 = (lo[a] - mv[a]) * inv, t2 = (hi[a] - mv[a]) * inv;
                        kmin = fmaxf(kmin, fminf(t1, t2) - 1.0f);
                        kmax = fminf(kmax, fmaxf(t1, t2) + 1.0f);
                    } else if (mv[a] < lo[a] || mv[a] > hi[a]) {
                        hit = false;
                    }
                }
                if (!hit || kmin > kmax) continue;
                const int i0 = max(static_cast<int>(ceilf(kmin - r.k0)), 0);
                const int i1 = min(static_cast<int>(floorf(kmax - r.k0)), r.n - 1);
                const float wgt = r.h * rv * inv_sub;
                for (int i = i0; i <= i1; ++i) {
                    const float kk = r.k0 + static_cast<float>(i);
                    float cx = fmaf(kk, r.hx, r.mx), cy = fmaf(kk, r.hy, r.my),
                          cz = fmaf(kk, r.hz, r.mz);
                    if (WARP && !warp(w, d, tau, cx, cy, cz)) continue;
                    int ix, iy, iz;
                    float fx, fy, fz;
                    corner_idx(d, cx, cy, cz, ix, iy, iz, fx, fy, fz);
                    const int lx = ix - x0, ly = iy - y0, lz = iz - z0;
                    const bool x_0 = lx >= 0 && lx < ex, x_1 = lx + 1 >= 0 && lx + 1 < ex;
                    const bool y_0 = ly >= 0 && ly < ey, y_1 = ly + 1 >= 0 && ly + 1 < ey;
                    const bool z_0 = lz >= 0 && lz < ez, z_1 = lz + 1 >= 0 && lz + 1 < ez;
                    if (!((x_0 || x_1) && (y_0 || y_1) && (z_0 || z_1))) continue;
                    const float gx1 = fx, gx0 = 1.0f - fx;
                    const float gy1 = fy, gy0 = 1.0f - fy;
                    const float gz1 = fz * wgt, gz0 = (1.0f - fz) * wgt;
                    const float w00 = gz0 * gy0, w01 = gz0 * gy1, w10 = gz1 * gy0, w11 = gz1 * gy1;
                    const int base = lz * sz + ly * sy + lx;   // may be outside: guarded
                    double *ap = acc + base;
                    if (z_0 && y_0 && x_0) atomicAdd(ap, static_cast<double>(w00 * gx0));
                    if (z_0 && y_0 && x_1) atomicAdd(ap + 1, static_cast<double>(w00 * gx1));
                    if (z_0 && y_1 && x_0) atomicAdd(ap + sy, static_cast<double>(w01 * gx0));
                    if (z_0 && y_1 && x_1) atomicAdd(ap + sy + 1, static_cast<double>(w01 * gx1));
                    if (z_1 && y_0 && x_0) atomicAdd(ap + sz, static_cast<double>(w10 * gx0));
                    if (z_1 && y_0 && x_1) atomicAdd(ap + sz + 1, static_cast<double>(w10 * gx1));
                    if (z_1 && y_1 && x_0) atomicAdd(ap + sz + sy, static_cast<double>(w11 * gx0));
                    if (z_1 && y_1 && x_1) atomicAdd(ap + sz + sy + 1, static_cast<double>(w11 * gx1));
                }
            }
        }
    }
    __syncthreads();
    // ---- write the brick out (x fastest)
    const int nvox = ex * ey * ez;
    for (int i = threadIdx.x; i < nvox; i += BP_THREADS) {
        const int lz = i / (ex * ey);
        const int rem = i - lz * ex * ey;
        const int ly = rem / ex;
        const int lx = rem - ly * ex;
        float *dst = vol + (static_cast<size_t>(z0 + lz) * g.ny + (y0 + ly)) * g.nx + (x0 + lx);
        const float v = static_cast<float>(acc[lz * sz + ly * sy + lx]);
        if (bg.chunks > 1) {
            if (v != 0.0f) unsafeAtomicAdd(dst, v);
        } else if (bg.accumulate) {
            *dst += v;
        } else {
            *dst = v;
        }
    }
}

}  // namespace

hipError_t launch_back(const RayGrid &g, const WarpGrid &w, const double *Pmat, const void *sino,
                       int sino_dtype, float *vol, int accumulate, int mode, hipStream_t stream) {
    if (g.n_views <= 0) return hipSuccess;
    BrickGrid bg;
    bg.bx = min(32, g.nx);
    bg.by = min(15, g.ny);
    bg.bz = min(16, g.nz);
    // FP64 cells span two 4-byte banks: odd row stride and a plane stride of
    // 3 (mod 16) put neighbours along y, z and the diagonals in other banks
    bg.sy = bg.bx | 1;
    bg.sz = bg.sy * bg.by + ((3 - (bg.sy * bg.by) % 16) + 16) % 16;
    bg.nbx = (g.nx + bg.bx - 1) / bg.bx;
    bg.nby = (g.ny + bg.by - 1) / bg.by;
    bg.nbz = (g.nz + bg.bz - 1) / bg.bz;
    const long long bricks = static_cast<long long>(bg.nbx) * bg.nby * bg.nbz;
    // enough workgroups to fill 256 CUs a few times over, at least 4 views each
    long long want = (2048 + bricks - 1) / bricks;
    const long long max_chunks = (g.n_views + 3) / 4;
    if (want > max_chunks) want = max_chunks;
    if (want < 1) want = 1;
    bg.views_per_chunk = static_cast<int>((g.n_views + want - 1) / want);
    bg.chunks = (g.n_views + bg.views_per_chunk - 1) / bg.views_per_chunk;
    bg.total = static_cast<int>(bricks * bg.chunks);
    bg.accumulate = accumulate;
    if (bg.chunks > 1 && !accumulate) {
        // chunks add into the volume: clear it first
        hipError_t e = launch_fill_zero(vol, sizeof(float) * static_cast<size_t>(g.nx) * g.ny * g.nz,
                                        stream);
        if (e != hipSuccess) return e;
    }
    const int per = (bg.total + N_XCD - 1) / N_XCD;
    const dim3 grid(static_cast<unsigned>(per * N_XCD)), block(BP_THREADS);
    const size_t shmem = sizeof(double) * static_cast<size_t>(bg.sz) * bg.bz;
    const bool wp = w.U != nullptr;
    if (mode == BP_ONES) {
        if (wp)
            hipLaunchKernelGGL((bp_brick_kernel<float, BP_ONES, true>), grid, block, shmem, stream,
                               g, w, Pmat, nullptr, vol, bg);
        else
            hipLaunchKernelGGL((bp_brick_kernel<float, BP_ONES, false>), grid, block, shmem,
                               stream, g, w, Pmat, nullptr, vol, bg);
        return hipGetLastError();
    }
#define CTREX_BP(T)                                                                              \
    {                                                                                            \
        const T *sp = static_cast<const T *>(sino);                                              \
        if (wp)                                                                                  \
            hipLaunchKernelGGL((bp_brick_kernel<T, BP_PLAIN, true>), grid, block, shmem, stream, \
                               g, w, Pmat, sp, vol, bg);                                         \
        else                                                                                     \
            hipLaunchKernelGGL((bp_brick_kernel<T, BP_PLAIN, false>), grid, block, shmem,        \
                               stream, g, w, Pmat, sp, vol, bg);                                 \
        return hipGetLastError();                                                                \
    }
    switch (sino_dtype) {
        case F32: CTREX_BP(float)
        case BF16: CTREX_BP(bf16_t)
        case F16: CTREX_BP(_Float16)
        default: return hipErrorInvalidValue;
    }
#undef CTREX_BP
}

}  // namespace ctrex
