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
// voxels) held in LDS for a whole chunk of projections, accumulated as 64-bit
// fixed point with LDS integer atomics: on gfx950 these sustain about twenty
// times the lane rate of LDS FP32 atomic adds, and the sums are exact (so the
// result does not depend on the order of the atomics).  A scale bounded from
// max|r| puts the largest possible contribution at 2^30, so each one is a
// 32-bit integer (weights formed in FP32, rounded to the nearest unit) while the 64-bit sums cannot overflow.  For every
// (projection, sub-view) it bounds the detector pixels whose rays can reach
// the brick (the projection of the brick grown by one voxel and the warp
// bound), redoes those rays' FP64 set-up, clips their sample range to the
// grown brick, and adds its eight corners with LDS 64-bit integer atomics.
// The LDS brick carries one halo cell on each side in x and y, which takes
// the corners that fall outside the brick there and is never written out; a
// corner outside in z gets weight zero.  A sample whose corner cube straddles
// a brick face is visited by each brick it touches, and each keeps only its
// own corners, so every corner is counted once.  There is no global atomic
// and no barrier inside the projection loop; the brick is written out once
// at the end (into a partial volume per projection chunk, summed in a fixed
// order, when several chunks share a brick).

#include "ray_common.h"

#include <type_traits>

namespace ctrex {
namespace {

using namespace dev;

// Launch shape.  Unwarped: 16 waves per workgroup, one workgroup per CU (its
// LDS brick and its waves' ray tables take 140 KB of the 160), so 4 waves per
// SIMD at up to 128 registers, with no spills.  The kernel is bound by LDS
// instructions, each taking about six CU cycles whatever its number of active
// lanes, so a hand-over reads the next ray from the table (four 16-byte reads
// by the lanes that hand over) instead of fifteen full-wave permutes.  Warped:
// the displacement lookups need the latency hiding of 6 waves per SIMD (12
// waves per workgroup, two per CU, no table), and hand-overs permute.
template <bool WARP> constexpr int bp_threads() { return WARP ? 768 : 1024; }
template <bool WARP> constexpr bool bp_table() { return !WARP; }

// Largest brick, and its LDS layout: rows of BRICK_X + 2 cells (halo on both
// sides, padded to an odd stride) and planes of BRICK_Y + 2 rows.  64-bit
// cells span two 4-byte banks; the odd row stride and a plane stride of 3
// (mod 16) put neighbours along y, z and the diagonals in other banks.  Two
// bricks (2 x 76 KB) share a CU's 160 KB of LDS.
constexpr int BRICK_X = 32, BRICK_Y = 15, BRICK_Z = 16;
constexpr int LDS_SY = (BRICK_X + 2) | 1;
constexpr int LDS_SZ = LDS_SY * (BRICK_Y + 2);
constexpr int LDS_CELLS = LDS_SZ * BRICK_Z;
static_assert(LDS_SZ % 16 == 3, "plane stride");

// Owner-computes bricks (the default form): a brick takes exactly the
// samples whose lower corner lies in it, so every sample is walked once and
// issues its eight atomics once, into LDS cells for the brick's voxels plus
// one halo layer on the high side of each axis (33 x 17 x 17 cells, 76.3 KB;
// row and plane strides 1 mod 16).  Every brick then adds its cells, halo
// included, into a 64-bit integer volume with global atomics; integer sums
// are exact, so neighbours' halos and projection chunks combine in any order
// and the result stays bitwise reproducible.  All workgroups use one
// fixed-point scale for that.  The direct form above (a sample walked by every
// brick it touches, each brick writing only its own voxels) needs no
// volume-sized buffer and serves the allocation-free entry point.
constexpr int OWN_X = 32, OWN_Y = 16, OWN_Z = 16;
constexpr int OWN_SY = OWN_X + 1;
constexpr int OWN_SZ = OWN_SY * (OWN_Y + 1);
constexpr int OWN_CELLS = OWN_SZ * (OWN_Z + 1);
constexpr int MAX_CELLS = OWN_CELLS > LDS_CELLS ? OWN_CELLS : LDS_CELLS;
static_assert(OWN_SY % 16 == 1 && OWN_SZ % 16 == 1, "owner strides");

struct BrickGrid {
    int bx, by, bz;       // brick size (voxels), at most BRICK_X x BRICK_Y x BRICK_Z
    int nbx, nby, nbz;    // bricks per axis
    int chunks;           // projection chunks per brick
    int views_per_chunk;
    int total;            // nbx * nby * nbz * chunks
    int accumulate;       // add into vol (else overwrite; needs chunks == 1)
    float wscale;         // every contribution is multiplied by this factor
    double cube_samples;  // max samples of one ray inside a side-2 cube
    float *partials;      // direct form: [chunks][nx*ny*nz] per-chunk results when chunks > 1
    unsigned long long *acc64;  // owner form: the 64-bit integer volume the bricks add into
};

// Fixed-point exponent of the owner form, the same in every workgroup and in
// the finishing pass: the largest contribution cmax at or below 2^30, and the
// sum into any voxel below 2^62 (at most every ray of every listed sub-view
// passes through the voxel's corner cube, each with at most cube_samples
// samples there).
__device__ __forceinline__ int own_kexp(double cmax, const RayGrid &g, double cube_samples) {
    const double rays = static_cast<double>(g.n_views) * g.n_sub * g.n_u * g.n_v;
    return static_cast<int>(floor(fmin(30.0 - log2(cmax), 62.0 - log2(rays * cube_samples * cmax))));
}

// A lane merges at most OWN_MERGE_MAX samples into its register sums (it
// starts a new run every OWN_MERGE_MAX iterations), and only while the sum of their ray weights |c| (each bounds all eight corner
// contributions of a sample, the trilinear weights being at most 1) stays at
// or below OWN_MERGE_LIMIT: the FP32 sums then exceed the exact ones by at
// most (1024 + 4) 2^-24 of 2^31 < 2^18, inside the 2^19 margin, so a merged
// corner sum converts to a 32-bit integer.
constexpr int OWN_MERGE_MAX = 1024;
static_assert((OWN_MERGE_MAX & (OWN_MERGE_MAX - 1)) == 0, "power of two");
constexpr float OWN_MERGE_LIMIT = 2147483648.0f - 524288.0f;   // 2^31 - 2^19

// Largest contribution of one sample to one corner: step * max|r| / n_sub
// times the caller's factor (and a margin for FP32 rounding).
__device__ __forceinline__ double contribution_bound(const RayGrid &g, double rmax, float wscale) {
    return rmax * g.step * (1.0 + 1e-5) * fabs(static_cast<double>(wscale)) / g.n_sub;
}

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

// Wave-uniform values computed by vector instructions (LDS reads, FP64 or
// float conversions) stay in vector registers unless moved to scalar ones;
// at 64 vector registers per lane they would be spilled.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uni(double x) {
    const long long b = __double_as_longlong(x);
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(b)));
    const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | lo);
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP lane moves:
// shifts by 1, 2, 4, 8 within each row of 16 lanes (zero shifted in), then
// the last lane of row 0 added to row 1 and of row 2 to row 3 (row broadcast
// 15), then lane 31 added to rows 2 and 3 (row broadcast 31).  No LDS and no
// per-lane addresses.  Called with all 64 lanes of the wave active.
__device__ __forceinline__ int wave_inclusive_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15 -> rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31 -> rows 2, 3
    return x;
}

// One contribution as a 64-bit fixed-point integer: c (FP32, the scale
// folded in, |c| < 2^31) rounded to the nearest integer, then sign-extended.
// Rounding errs by at most half a unit and without bias, so the error of a
// voxel's sum grows with the square root of its number of contributions.
__device__ __forceinline__ unsigned long long to_fixed(float c) {
    return static_cast<unsigned long long>(static_cast<long long>(static_cast<int>(rintf(c))));
}

// One ray of a wave's 8x8 pixel block, as the lanes that walk its samples
// need it: position of its first sample in the brick range and its step (both
// 64-bit fixed point), its weight, the end of its samples in the wave's order
// and the next ray of the block with samples (64 bytes, four 16-byte reads).
struct alignas(16) RayRec {
    long long px, py, pz;
    long long tx, ty, tz;
    float wq;
    int end;
    int next;
    int pad;
};
static_assert(sizeof(RayRec) == 64, "ray record");

// Orders one wave's LDS writes before its other lanes' reads of them (and
// those reads before the next writes); no instruction beyond a wait.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename TS, int MODE, bool WARP, bool OWN>
__global__ __launch_bounds__(bp_threads<WARP>())
__attribute__((amdgpu_waves_per_eu(WARP ? 6 : 4, WARP ? 6 : 4))) void bp_brick_kernel(RayGrid g, WarpGrid w,
                                                              const double *__restrict__ Pmat,
                                                              const TS *__restrict__ sino,
                                                              const float *__restrict__ rmax,
                                                              float *__restrict__ vol,
                                                              BrickGrid bg) {
    __shared__ unsigned long long acc[MAX_CELLS];
    constexpr int BP_THREADS = bp_threads<WARP>();
    constexpr bool TABLE = bp_table<WARP>();
    __shared__ double red[BP_THREADS / 64];
    __shared__ RayRec rays[TABLE ? BP_THREADS : 1];
    RayRec *const tabw = rays + (threadIdx.x & ~63);
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
    const int nlds = OWN ? OWN_CELLS : LDS_SZ * ez;
    for (int i = threadIdx.x; i < nlds; i += BP_THREADS) acc[i] = 0ull;
    // cell (lx, ly, lz) of the brick: direct form lx in [-1, ex], ly in
    // [-1, ey]; owner form lx in [0, ex], ly in [0, ey], lz in [0, ez]
    unsigned long long *const cell0 = OWN ? acc : acc + LDS_SY + 1;

    const VolDims d = vol_dims(g);
    const float M = static_cast<float>(w.margin);
    // samples with an (unwarped) position in [lo, hi] can touch the brick,
    // for any projection (the warp bound of the whole scan)
    const double lod[3] = {x0 - 1.0 - M, y0 - 1.0 - M, z0 - 1.0 - M};
    const double hid[3] = {static_cast<double>(x0 + ex) + M, static_cast<double>(y0 + ey) + M,
                           static_cast<double>(z0 + ez) + M};
    const double off[3] = {0.5 * (g.nx - 1), 0.5 * (g.ny - 1), 0.5 * (g.nz - 1)};
    // 1 / n_sub and the caller's factor (1 unless scaled; exact when a power of 2)
    const float inv_sub = uni(bg.wscale / static_cast<float>(g.n_sub));
    // largest side times 2^-22: four times the FP32 rounding error of a
    // coordinate of a ray's start
    const float tol = uni(static_cast<float>(max(g.nx, max(g.ny, g.nz))) * 2.38418579e-7f);
    const int k_first = chunk * bg.views_per_chunk;
    const int k_end = min(k_first + bg.views_per_chunk, g.n_views);
    const int n_pairs = (k_end - k_first) * g.n_sub;

    // ---- fixed-point scale.  Each contribution is at most
    // cmax = step * max|r| / n_sub (times the caller's factor), and every
    // contribution to a voxel comes from a sample of a ray in some pair's
    // pixel box lying in the voxel's corner cube (side 2), at most
    // bg.cube_samples of them per ray.  The scale 2^kexp puts the largest
    // contribution at or below 2^30 (so it fits a 32-bit integer) and keeps
    // the bound on the sums below 2^62.
    double nrays = 0.0;
    for (int q = threadIdx.x; q < (OWN ? 0 : n_pairs); q += BP_THREADS) {
        const int k = k_first + q / g.n_sub;
        const int p = g.views ? g.views[k] : k;
        const int sv_idx = p * g.n_sub + q % g.n_sub;
        int u0, u1, v0, v1;
        if (project_box(Pmat + 12 * static_cast<size_t>(sv_idx), lod, hid, off, g.n_u, g.n_v, u0,
                        u1, v0, v1))
            nrays += (u0 <= u1 && v0 <= v1) ? double(u1 - u0 + 1) * double(v1 - v0 + 1) : 0.0;
        else
            nrays += double(g.n_u) * double(g.n_v);
    }
    for (int o = 32; o > 0; o >>= 1) nrays += __shfl_xor(nrays, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrays;
    __syncthreads();
    nrays = 0.0;
    for (int i = 0; i < BP_THREADS / 64; ++i) nrays += red[i];
    const double cmax =
        contribution_bound(g, (MODE == BP_ONES) ? 1.0 : static_cast<double>(*rmax), bg.wscale);
    const double bound = OWN ? cmax : nrays * bg.cube_samples * cmax;
    const bool bad = !(cmax < __builtin_inf());   // NaN or Inf in the input: propagate NaN
    const bool any = uni(static_cast<int>(bound > 0.0 && !bad)) != 0;
    const int kexp = uni(!any ? 0
                         : OWN ? own_kexp(cmax, g, bg.cube_samples)
                               : static_cast<int>(floor(fmin(30.0 - log2(cmax),
                                                             62.0 - log2(bound)))));
    const double scale = uni(ldexp(1.0, kexp));

    // each wave takes whole (projection, sub-view) pairs, so a pair's pixel
    // box is projected once, by the wave that walks its rays
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    for (int q = wave; q < n_pairs && any; q += BP_THREADS / 64) {
        const int k = k_first + q / g.n_sub;
        const int s = q - (q / g.n_sub) * g.n_sub;
        const int p = uni(g.views ? g.views[k] : k);
        {
            const int sv_idx = p * g.n_sub + s;
            const SubView &sv = g.tab[sv_idx];
            // this sub-view's warp moves samples by at most |tau| max|U| on
            // every axis: its samples within that margin of the brick can
            // touch it (time-linear fields: half the scan's bound on average)
            const double mv = WARP ? fabs(sv.tau) * w.umax : 0.0;
            const float Mp = uni(mv > 0.0 ? static_cast<float>(ceil(mv * (1.0 + 1e-6) + 1e-6)) : 0.0f);
            // direct form: samples with a corner in the brick, position in
            // [x0 - 1, x0 + ex]; owner form: lower corner in it, [x0, x0 + ex]
            // The ray-range estimate below takes the ray's start in FP32,
            // off by up to 2^-24 of a coordinate: the bounds are widened by
            // 2^-22 of the largest side (this adds samples that the
            // exact corner test then rejects; for a ray almost parallel to an
            // axis the one-sample widening would not cover it)
            const float g0 = (OWN ? 0.0f : 1.0f) + tol;
            const float lo[3] = {uni(x0 - g0 - Mp), uni(y0 - g0 - Mp), uni(z0 - g0 - Mp)};
            const float hi[3] = {uni(static_cast<float>(x0 + ex) + Mp + tol),
                                 uni(static_cast<float>(y0 + ey) + Mp + tol),
                                 uni(static_cast<float>(z0 + ez) + Mp + tol)};
            const double plo[3] = {lo[0], lo[1], lo[2]}, phi[3] = {hi[0], hi[1], hi[2]};
            int u0 = 0, u1 = g.n_u - 1, v0 = 0, v1 = g.n_v - 1;
            if (!project_box(Pmat + 12 * static_cast<size_t>(sv_idx), plo, phi, off, g.n_u, g.n_v,
                             u0, u1, v0, v1)) {
                u0 = 0;
                u1 = g.n_u - 1;
                v0 = 0;
                v1 = g.n_v - 1;
            }
            u0 = uni(u0);
            u1 = uni(u1);
            v0 = uni(v0);
            v1 = uni(v1);
            if (u0 > u1 || v0 > v1) continue;
            // rays in 8x8 pixel blocks, one block per pass; the wave shares
            // each block's samples evenly among its lanes
            const int bu = (u1 - u0 + 8) >> 3;
            const int nblk = bu * ((v1 - v0 + 8) >> 3);
            const float tau = uni(static_cast<float>(sv.tau));
            const int lane = threadIdx.x & 63;
            for (int blk = 0; blk < nblk; ++blk) {
                const int iv = v0 + (blk / bu) * 8 + (lane >> 3);
                const int iu = u0 + (blk % bu) * 8 + (lane & 7);
                // ---- this lane's ray: its samples that can reach the brick
                int len = 0, ib = 0;
                float wq = 0.0f;   // h r / n_sub in fixed-point units
                Ray r;
                r.qx = r.qy = r.qz = r.tx = r.ty = r.tz = 0;
                const float rv = (iu > u1 || iv > v1) ? 0.0f
                                 : (MODE == BP_ONES) ? 1.0f
                                                     : ld(sino, (k * g.n_v + iv) * g.n_u + iu);
                if (rv != 0.0f && setup_ray(sv, static_cast<double>(iu), static_cast<double>(iv),
                                            g.nx, g.ny, g.nz, g.step, r)) {
                    // sample indices i with b + i s inside [lo, hi] on every
                    // axis, in FP32 (corners are checked exactly below).  The
                    // FP32 start and step put b + i s within 2^-24 (|b| + L) <
                    // 2.8 2^-24 max side of the fixed-point position of sample
                    // i (L the ray length, at most sqrt(3) max side), and
                    // [lo, hi] is widened by tol = 4 2^-24 max side; the index estimate itself is three
                    // roundings, under 3 2^-24 |t|, inside the margin of
                    // 1/64 + 2^-20 |t| samples.  An axis the ray does not move
                    // along (|s| under 1e-30: its samples drift by less than
                    // tol) only decides whether the ray hits; branch-free.
                    float kmin = 0.0f, kmax = static_cast<float>(r.n - 1);
                    const float bv[3] = {r.bx, r.by, r.bz};
                    const float sv3[3] = {r.fx, r.fy, r.fz};
                    bool hit = true;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const bool flat = fabsf(sv3[q]) < 1e-30f;
                        const float inv = 1.0f / (flat ? 1.0f : sv3[q]);
                        const float t1 = (lo[q] - bv[q]) * inv, t2 = (hi[q] - bv[q]) * inv;
                        const float tl = fminf(t1, t2), th = fmaxf(t1, t2);
                        const float ml = fmaf(fabsf(tl), 9.5367431640625e-7f, 0.015625f);
                        const float mh = fmaf(fabsf(th), 9.5367431640625e-7f, 0.015625f);
                        kmin = flat ? kmin : fmaxf(kmin, tl - ml);
                        kmax = flat ? kmax : fminf(kmax, th + mh);
                        hit &= !(flat & ((bv[q] < lo[q]) | (bv[q] > hi[q])));
                    }
                    if (hit && kmin <= kmax) {
                        ib = max(static_cast<int>(ceilf(kmin)), 0);
                        const int ie = min(static_cast<int>(floorf(kmax)), r.n - 1);
                        len = max(ie - ib + 1, 0);
                        wq = static_cast<float>(static_cast<double>(r.h * rv * inv_sub) * scale);
                    }
                }
                // ---- exclusive prefix of the segment lengths over the wave
                const int incl = wave_inclusive_sum(len);
                const int S = incl - len;
                const int T = __builtin_amdgcn_readlane(incl, 63);
                if (T == 0) continue;   // uniform over the wave
                const unsigned long long live = __ballot(len > 0);
                // ---- this lane's ray (position of its first sample in the
                // brick range, step, weight, end of its samples in the wave's
                // order, next ray with samples) for the lanes that walk into
                // it: in the wave's LDS table, or permuted from this lane
                RayRec mine;
                {
                    const unsigned long long later =
                        lane < 63 ? (live & (~0ull << (lane + 1))) : 0ull;
                    mine.px = r.qx + static_cast<long long>(ib) * r.tx;
                    mine.py = r.qy + static_cast<long long>(ib) * r.ty;
                    mine.pz = r.qz + static_cast<long long>(ib) * r.tz;
                    mine.tx = r.tx;
                    mine.ty = r.ty;
                    mine.tz = r.tz;
                    mine.wq = wq;
                    mine.end = incl;
                    mine.next = later ? __ffsll(static_cast<long long>(later)) - 1 : lane;
                    mine.pad = 0;
                }
                // the record of ray `src` (every lane executes the permutes: a
                // permute skipped by the source lane returns 0)
                auto fetch = [&](int src) {
                    RayRec e;
                    if (TABLE) {
                        e = tabw[src];
                    } else {
                        e.px = __shfl(mine.px, src, 64);
                        e.py = __shfl(mine.py, src, 64);
                        e.pz = __shfl(mine.pz, src, 64);
                        e.tx = __shfl(mine.tx, src, 64);
                        e.ty = __shfl(mine.ty, src, 64);
                        e.tz = __shfl(mine.tz, src, 64);
                        e.wq = __shfl(mine.wq, src, 64);
                        e.end = __shfl(mine.end, src, 64);
                        e.next = __shfl(mine.next, src, 64);
                    }
                    return e;
                };
                if (TABLE) {
                    tabw[lane] = mine;
                    wave_sync();
                }
                // ---- lane takes samples [start, end) of the wave's T
                const int start = (T * lane) >> 6, end = (T * (lane + 1)) >> 6;
                int j = 0;   // last ray with S_j <= start: it owns sample `start`
#pragma unroll
                for (int st = 32; st > 0; st >>= 1) {
                    const int t = j + st;
                    if (__shfl(S, t, 64) <= start) j = t;
                }
                // the lane's first ray may be entered mid-way: `start - S_j`
                // samples after its first sample in the brick range
                const long long m = start - __shfl(S, j, 64);
                long long px, py, pz, ctx, cty, ctz;
                float cwq;
                int cend, cnext;
                {
                    const RayRec e = fetch(j);
                    ctx = e.tx;
                    cty = e.ty;
                    ctz = e.tz;
                    px = e.px + m * ctx;
                    py = e.py + m * cty;
                    pz = e.pz + m * ctz;
                    cwq = e.wq;
                    cend = e.end;
                    cnext = e.next;
                }
                const int trips = (T + 63) >> 6;
                // the sample walk, with the corner clamps (CLAMP) or without:
                // in the unwarped owner form a brick that holds neither the
                // first lower corner 0 nor the last two n - 2, n - 1 on any
                // axis needs none, since a sample the clamp would move has its
                // lower corner outside the brick before and after the clamp
                auto walk = [&](auto clamp_tag) {
                    constexpr bool CLAMP = decltype(clamp_tag)::value;
                    // owner form: each lane keeps the eight corner sums of the
                    // cell its last samples fell in and adds them to LDS only
                    // when the next sample falls in another cell (consecutive
                    // samples 0.5 voxel apart often share one), when another
                    // sample could take a sum past a 32-bit integer, or every
                    // OWN_MERGE_MAX iterations; the sums are flushed at the end
                    // of the block, so they hold no registers during the next
                    // block's ray set-up
                    int mcell = -1;
                    float msum = 0.0f;
                    float m0 = 0.0f, m1 = 0.0f, m2 = 0.0f, m3 = 0.0f;
                    float m4 = 0.0f, m5 = 0.0f, m6 = 0.0f, m7 = 0.0f;
                    auto flush = [&]() {
                        unsigned long long *const f0 = cell0 + mcell;
                        unsigned long long *const f1 = f0 + OWN_SZ;
                        atomicAdd(f0, to_fixed(m0));
                        atomicAdd(f0 + 1, to_fixed(m1));
                        atomicAdd(f0 + OWN_SY, to_fixed(m2));
                        atomicAdd(f0 + OWN_SY + 1, to_fixed(m3));
                        atomicAdd(f1, to_fixed(m4));
                        atomicAdd(f1 + 1, to_fixed(m5));
                        atomicAdd(f1 + OWN_SY, to_fixed(m6));
                        atomicAdd(f1 + OWN_SY + 1, to_fixed(m7));
                    };
                    int pos = start;
                    for (int it = 0; it < trips; ++it) {
                        // wave-uniform hand-over to the next ray with samples;
                        // it is entered at its first sample in the brick range
                        const bool need = pos < end && pos == cend;
                        if (TABLE ? need : __any(need)) {
                            // with the table only the lanes that hand over
                            // read; permutes run on every lane, and the others
                            // keep their ray
                            const RayRec f = fetch(TABLE ? cnext : (need ? cnext : lane));
                            const RayRec e = need ? f : RayRec{px, py, pz, ctx, cty, ctz,
                                                               cwq, cend, cnext, 0};
                            px = e.px;
                            py = e.py;
                            pz = e.pz;
                            ctx = e.tx;
                            cty = e.ty;
                            ctz = e.tz;
                            cwq = e.wq;
                            cend = e.end;
                            cnext = e.next;
                        }
                        if (pos >= end) continue;
                        ++pos;
                        const long long qx = px, qy = py, qz = pz;
                        px += ctx;
                        py += cty;
                        pz += ctz;
                        int ix, iy, iz;
                        float fx, fy, fz;
                        if (CLAMP || WARP) {
                            if (!sample_corner<WARP>(d, w, tau, qx, qy, qz, ix, iy, iz, fx, fy, fz))
                                continue;
                        } else {
                            fx_split(qx, ix, fx);
                            fx_split(qy, iy, fy);
                            fx_split(qz, iz, fz);
                        }
                        const int lx = ix - x0, ly = iy - y0, lz = iz - z0;
                        if (OWN) {
                            // another brick owns this sample's lower corner
                            if (static_cast<uint32_t>(lx) >= static_cast<uint32_t>(ex) ||
                                static_cast<uint32_t>(ly) >= static_cast<uint32_t>(ey) ||
                                static_cast<uint32_t>(lz) >= static_cast<uint32_t>(ez))
                                continue;
                            const float gx1 = fx, gx0 = 1.0f - fx;
                            const float gy1 = fy, gy0 = 1.0f - fy;
                            const float gz1 = fz * cwq, gz0 = (1.0f - fz) * cwq;
                            const float w00 = gz0 * gy0, w01 = gz0 * gy1, w10 = gz1 * gy0,
                                        w11 = gz1 * gy1;
                            const int cell = __mul24(lz, OWN_SZ) + __mul24(ly, OWN_SY) + lx;
                            if (WARP) {
                                // warped samples change cells too often for
                                // the merge to pay (measured 6 % slower):
                                // add every sample at once
                                unsigned long long *const a0 = cell0 + cell;
                                unsigned long long *const a1 = a0 + OWN_SZ;
                                atomicAdd(a0, to_fixed(w00 * gx0));
                                atomicAdd(a0 + 1, to_fixed(w00 * gx1));
                                atomicAdd(a0 + OWN_SY, to_fixed(w01 * gx0));
                                atomicAdd(a0 + OWN_SY + 1, to_fixed(w01 * gx1));
                                atomicAdd(a1, to_fixed(w10 * gx0));
                                atomicAdd(a1 + 1, to_fixed(w10 * gx1));
                                atomicAdd(a1 + OWN_SY, to_fixed(w11 * gx0));
                                atomicAdd(a1 + OWN_SY + 1, to_fixed(w11 * gx1));
                                continue;
                            }
                            const float aw = fabsf(cwq);
                            const bool fresh = (it & (OWN_MERGE_MAX - 1)) == 0;   // uniform
                            const bool same =
                                !fresh && cell == mcell && msum + aw <= OWN_MERGE_LIMIT;
                            if (!same && mcell >= 0) flush();
                            const float k0 = same ? m0 : 0.0f, k1 = same ? m1 : 0.0f;
                            const float k2 = same ? m2 : 0.0f, k3 = same ? m3 : 0.0f;
                            const float k4 = same ? m4 : 0.0f, k5 = same ? m5 : 0.0f;
                            const float k6 = same ? m6 : 0.0f, k7 = same ? m7 : 0.0f;
                            m0 = fmaf(w00, gx0, k0);
                            m1 = fmaf(w00, gx1, k1);
                            m2 = fmaf(w01, gx0, k2);
                            m3 = fmaf(w01, gx1, k3);
                            m4 = fmaf(w10, gx0, k4);
                            m5 = fmaf(w10, gx1, k5);
                            m6 = fmaf(w11, gx0, k6);
                            m7 = fmaf(w11, gx1, k7);
                            msum = same ? msum + aw : aw;
                            mcell = cell;
                            continue;
                        }
                        // no corner in the brick: lx, ly outside [-1, e - 1] (the
                        // halo takes -1 and e - 1's upper neighbour), or lz
                        // outside [-1, ez - 1]
                        if (static_cast<uint32_t>(lx + 1) > static_cast<uint32_t>(ex) ||
                            static_cast<uint32_t>(ly + 1) > static_cast<uint32_t>(ey) ||
                            static_cast<uint32_t>(lz + 1) > static_cast<uint32_t>(ez))
                            continue;
                        const bool z_0 = lz >= 0, z_1 = lz + 1 < ez;
                        // corner weights in FP32 with the ray weight and the
                        // fixed-point scale folded in; each contribution becomes a
                        // 32-bit integer added into the 64-bit cell.  x and y
                        // neighbours outside the brick land in the halo; a z
                        // neighbour outside gets weight zero and a plane clamped
                        // into the brick (adding an integer zero changes no sum),
                        // so every lane issues the same eight atomics.
                        const float gx1 = fx, gx0 = 1.0f - fx;
                        const float gy1 = fy, gy0 = 1.0f - fy;
                        const float gz1 = (z_1 ? fz : 0.0f) * cwq;
                        const float gz0 = (z_0 ? 1.0f - fz : 0.0f) * cwq;
                        const float w00 = gz0 * gy0, w01 = gz0 * gy1, w10 = gz1 * gy0,
                                    w11 = gz1 * gy1;
                        const int row = __mul24(ly, LDS_SY) + lx;
                        unsigned long long *const a0 = cell0 + (__mul24(max(lz, 0), LDS_SZ) + row);
                        unsigned long long *const a1 =
                            cell0 + (__mul24(min(lz + 1, ez - 1), LDS_SZ) + row);
                        atomicAdd(a0, to_fixed(w00 * gx0));
                        atomicAdd(a0 + 1, to_fixed(w00 * gx1));
                        atomicAdd(a0 + LDS_SY, to_fixed(w01 * gx0));
                        atomicAdd(a0 + LDS_SY + 1, to_fixed(w01 * gx1));
                        atomicAdd(a1, to_fixed(w10 * gx0));
                        atomicAdd(a1 + 1, to_fixed(w10 * gx1));
                        atomicAdd(a1 + LDS_SY, to_fixed(w11 * gx0));
                        atomicAdd(a1 + LDS_SY + 1, to_fixed(w11 * gx1));
                    }
                    if (OWN && !WARP && mcell >= 0) flush();
                };
                const bool interior = OWN && !WARP && x0 >= 1 && x0 + ex <= g.nx - 2 && y0 >= 1 &&
                                      y0 + ey <= g.ny - 2 && z0 >= 1 && z0 + ez <= g.nz - 2;
                if (interior)
                    walk(std::false_type{});
                else
                    walk(std::true_type{});
                if (TABLE) wave_sync();   // the table is rewritten by the next block
            }
        }
    }
    __syncthreads();
    if (OWN) {
        // ---- add the brick's cells, halo included, into the integer volume
        for (int i = threadIdx.x; i < OWN_CELLS; i += BP_THREADS) {
            const int lz = i / OWN_SZ;
            const int rem = i - lz * OWN_SZ;
            const int ly = rem / OWN_SY;
            const int lx = rem - ly * OWN_SY;
            const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
            const unsigned long long q = acc[i];
            if (q != 0ull && lx <= ex && ly <= ey && lz <= ez && gx < g.nx && gy < g.ny &&
                gz < g.nz)
                atomicAdd(bg.acc64 + (static_cast<size_t>(gz) * g.ny + gy) * g.nx + gx, q);
        }
        return;
    }
    // ---- write the brick out (x fastest)
    const double inv_scale = ldexp(1.0, -kexp);
    const int nvox = ex * ey * ez;
    for (int i = threadIdx.x; i < nvox; i += BP_THREADS) {
        const int lz = i / (ex * ey);
        const int rem = i - lz * ex * ey;
        const int ly = rem / ex;
        const int lx = rem - ly * ex;
        float *dst = vol + (static_cast<size_t>(z0 + lz) * g.ny + (y0 + ly)) * g.nx + (x0 + lx);
        const long long q = static_cast<long long>(cell0[lz * LDS_SZ + ly * LDS_SY + lx]);
        const float v = bad ? __builtin_nanf("") : static_cast<float>(static_cast<double>(q) * inv_scale);
        if (bg.chunks > 1) {
            // each chunk owns a slab; a fixed-order sum combines them
            bg.partials[static_cast<size_t>(chunk) * g.nx * g.ny * g.nz + (dst - vol)] = v;
        } else if (bg.accumulate) {
            *dst += v;
        } else {
            *dst = v;
        }
    }
}

// vol[i] (+)= sum over chunks c of part[c][i], in chunk order.
__global__ __launch_bounds__(256) void sum_chunks_kernel(const float *__restrict__ part, int chunks,
                                                         size_t n, int accumulate,
                                                         float *__restrict__ vol) {
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
        float s = accumulate ? vol[i] : 0.0f;
        for (int c = 0; c < chunks; ++c) s += part[static_cast<size_t>(c) * n + i];
        vol[i] = s;
    }
}

// Owner form: vol[i] = (vol[i] if accumulate) + acc64[i] 2^-kexp, NaN for a
// non-finite max |r|, with the exponent every brick used.
template <int MODE>
__global__ __launch_bounds__(256) void own_finish_kernel(const unsigned long long *__restrict__ acc64,
                                                         size_t n, const float *__restrict__ rmax,
                                                         RayGrid g, double cube_samples,
                                                         float wscale, int accumulate,
                                                         float *__restrict__ vol) {
    const double cmax =
        contribution_bound(g, MODE == BP_ONES ? 1.0 : static_cast<double>(*rmax), wscale);
    const bool bad = !(cmax < __builtin_inf());
    const double inv = (cmax > 0.0 && !bad) ? ldexp(1.0, -own_kexp(cmax, g, cube_samples)) : 0.0;
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
        const float v = bad ? __builtin_nanf("")
                            : static_cast<float>(static_cast<double>(static_cast<long long>(acc64[i])) * inv);
        vol[i] = accumulate ? vol[i] + v : v;
    }
}

BrickGrid plan_bricks(const RayGrid &g, int cap_chunks, bool own) {
    BrickGrid bg;
    bg.bx = min(own ? OWN_X : BRICK_X, g.nx);
    bg.by = min(own ? OWN_Y : BRICK_Y, g.ny);
    bg.bz = min(own ? OWN_Z : BRICK_Z, g.nz);
    bg.nbx = (g.nx + bg.bx - 1) / bg.bx;
    bg.nby = (g.ny + bg.by - 1) / bg.by;
    bg.nbz = (g.nz + bg.bz - 1) / bg.bz;
    const long long bricks = static_cast<long long>(bg.nbx) * bg.nby * bg.nbz;
    // enough workgroups to fill 256 CUs a few times over, at least 4 views each
    long long want = (2048 + bricks - 1) / bricks;
    const long long max_chunks = (g.n_views + 3) / 4;
    if (want > max_chunks) want = max_chunks;
    if (cap_chunks > 0 && want > cap_chunks) want = cap_chunks;
    if (want < 1) want = 1;
    bg.views_per_chunk = static_cast<int>((g.n_views + want - 1) / want);
    bg.chunks = (g.n_views + bg.views_per_chunk - 1) / bg.views_per_chunk;
    bg.total = static_cast<int>(bricks * bg.chunks);
    // h >= step / 2 whenever a ray has two samples, and a side-2 cube holds a
    // chord of at most 2 sqrt(3)
    bg.cube_samples = floor(4.0 * 1.7320508075688772 / g.step) + 1.0;
    bg.partials = nullptr;
    bg.acc64 = nullptr;
    bg.accumulate = 0;
    bg.wscale = 1.0f;
    return bg;
}

}  // namespace

size_t back_scratch_bytes(const RayGrid &g, int max_chunks, bool direct) {
    if (g.n_views <= 0) return 0;
    const size_t nvol = static_cast<size_t>(g.nx) * g.ny * g.nz;
    if (!direct) return sizeof(unsigned long long) * nvol;
    const BrickGrid bg = plan_bricks(g, max_chunks, false);
    return bg.chunks > 1 ? sizeof(float) * static_cast<size_t>(bg.chunks) * nvol : 0;
}

hipError_t launch_back(const RayGrid &g, const WarpGrid &w, const double *Pmat, const void *sino,
                       int sino_dtype, float *vol, int accumulate, int mode, float *scratch,
                       void *work, hipStream_t stream, float scale, int max_chunks, bool direct) {
    if (g.n_views <= 0) return hipSuccess;
    BrickGrid bg = plan_bricks(g, direct ? max_chunks : 0, !direct);
    bg.accumulate = accumulate;
    bg.wscale = scale;
    const size_t nvol = static_cast<size_t>(g.nx) * g.ny * g.nz;
    if (direct) {
        bg.partials = static_cast<float *>(work);
        if (bg.chunks > 1 && !work) return hipErrorInvalidValue;
    } else {
        bg.acc64 = static_cast<unsigned long long *>(work);
        if (!work) return hipErrorInvalidValue;
        hipError_t e = launch_fill_zero(work, sizeof(unsigned long long) * nvol, stream);
        if (e != hipSuccess) return e;
    }
    const int per = (bg.total + N_XCD - 1) / N_XCD;
    const bool wp = w.U != nullptr;
    const dim3 grid(static_cast<unsigned>(per * N_XCD));
    const dim3 block(static_cast<unsigned>(wp ? bp_threads<true>() : bp_threads<false>()));
    const size_t shmem = 0;   // the brick is static LDS
    size_t fblocks = (nvol + 255) / 256;
    if (fblocks > 65536) fblocks = 65536;
    // after the bricks: the direct form's chunk partials summed in chunk
    // order, or the owner form's integer volume scaled into vol
    auto finish = [&](int m) -> hipError_t {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (!direct) {
            if (m == BP_ONES)
                hipLaunchKernelGGL(own_finish_kernel<BP_ONES>, dim3(static_cast<unsigned>(fblocks)),
                                   dim3(256), 0, stream, bg.acc64, nvol, scratch, g,
                                   bg.cube_samples, scale, accumulate, vol);
            else
                hipLaunchKernelGGL(own_finish_kernel<BP_PLAIN>,
                                   dim3(static_cast<unsigned>(fblocks)), dim3(256), 0, stream,
                                   bg.acc64, nvol, scratch, g, bg.cube_samples, scale, accumulate,
                                   vol);
            return hipGetLastError();
        }
        if (bg.chunks <= 1) return hipSuccess;
        hipLaunchKernelGGL(sum_chunks_kernel, dim3(static_cast<unsigned>(fblocks)), dim3(256), 0,
                           stream, bg.partials, bg.chunks, nvol, accumulate, vol);
        return hipGetLastError();
    };
#define CTREX_BP_LAUNCH(T, M, SP, RM)                                                           \
    {                                                                                           \
        if (direct) {                                                                           \
            if (wp)                                                                             \
                hipLaunchKernelGGL((bp_brick_kernel<T, M, true, false>), grid, block, shmem,    \
                                   stream, g, w, Pmat, SP, RM, vol, bg);                        \
            else                                                                                \
                hipLaunchKernelGGL((bp_brick_kernel<T, M, false, false>), grid, block, shmem,   \
                                   stream, g, w, Pmat, SP, RM, vol, bg);                        \
        } else {                                                                                \
            if (wp)                                                                             \
                hipLaunchKernelGGL((bp_brick_kernel<T, M, true, true>), grid, block, shmem,     \
                                   stream, g, w, Pmat, SP, RM, vol, bg);                        \
            else                                                                                \
                hipLaunchKernelGGL((bp_brick_kernel<T, M, false, true>), grid, block, shmem,    \
                                   stream, g, w, Pmat, SP, RM, vol, bg);                        \
        }                                                                                       \
        return finish(M);                                                                       \
    }
    if (mode == BP_ONES) CTREX_BP_LAUNCH(float, BP_ONES, nullptr, nullptr)
    // max |r| over the sinogram sets the fixed-point scale
    const size_t n_sino = static_cast<size_t>(g.n_views) * g.n_u * g.n_v;
    hipError_t e = launch_max_abs(sino, sino_dtype, n_sino, scratch, stream);
    if (e != hipSuccess) return e;
    switch (sino_dtype) {
        case F32: CTREX_BP_LAUNCH(float, BP_PLAIN, static_cast<const float *>(sino), scratch)
        case BF16: CTREX_BP_LAUNCH(bf16_t, BP_PLAIN, static_cast<const bf16_t *>(sino), scratch)
        case F16: CTREX_BP_LAUNCH(_Float16, BP_PLAIN, static_cast<const _Float16 *>(sino), scratch)
        default: return hipErrorInvalidValue;
    }
#undef CTREX_BP_LAUNCH
}

}  // namespace ctrex
