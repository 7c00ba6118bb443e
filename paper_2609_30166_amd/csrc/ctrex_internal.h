// Internal types shared by the host runtime and the HIP kernels of libctrex.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ctrex {

// Per sub-view geometry as the kernels read it (one 128-byte entry per
// (projection, sub-view)): source in index coordinates, inverse of the 3x3
// block of the view matrix, and the warp time fraction.  FP64 (Sec. 2.2).
struct alignas(16) SubView {
    double S[3];
    double Mi[9];
    double tau;
    double pad[3];
};
static_assert(sizeof(SubView) == 128, "SubView layout");

// Storage types (match CTREX_F32 / CTREX_BF16 / CTREX_F16).
enum DType : int { F32 = 0, BF16 = 1, F16 = 2 };

// 16-bit brain-float storage (top half of an IEEE float).
struct bf16_t {
    uint16_t bits;
};

struct RayGrid {
    const SubView *tab;  // [n_proj * n_sub]
    const int *views;    // device list of n_views projection indices, or nullptr
    int n_views;
    int n_sub;
    int n_u, n_v;
    int nx, ny, nz;
    double step;
    // detector tiling of the launch
    int tiles_u, tiles_v;
    int total_blocks;    // tiles_u * tiles_v * n_views
    int tube = 0;        // forward projection of FP32 volumes through LDS-staged tubes
};

struct WarpGrid {
    const float4 *U;     // repacked [gz][gy][gx] (x, y, z, 0), or nullptr
    int gx, gy, gz;
    double sx, sy, sz;   // index -> grid coordinate scale (g - 1) / (n - 1)
    float fsx, fsy, fsz; // the same scales in FP32 (used by the sample loops)
    int margin;          // whole voxels bounding |tau * U| on every axis
    double umax;         // max |U component| (a sub-view moves samples by <= |tau| umax)
};


// Forward-projection modes.
enum FpMode : int {
    FP_PLAIN = 0,     // sino = A vol
    FP_RECIP_ONES = 1,// out = 1 / (A 1), 0 where A 1 == 0 (the SIRT weight R)
    FP_CORRECT = 2,   // out = R (b - A vol); per-block sums of (b - A vol)^2
    FP_RESIDUAL = 3,  // per-block sums of (b - A vol)^2 only (out unused)
};

struct FpExtra {
    const void *b;       // measured sinogram (FP_CORRECT, FP_RESIDUAL), storage type = out type
    const float *R;      // detector weights (FP_CORRECT); nullptr: the constant rscale
    double *partials;    // [total_blocks] (FP_CORRECT, FP_RESIDUAL)
    float rscale = 1.0f; // FP_CORRECT without R: out = rscale (b - A vol)
    const void *vol_t = nullptr;  // optional y-fastest copy [nz][nx][ny] of the volume
    // optional corner-packed copies of an FP32 volume (element (x, y, z) = the
    // four corners v(x, y), v(x+1, y), v(x, y+1), v(x+1, y+1) of slice z):
    // x-fastest [nz][ny][nx] and y-fastest [nz][nx][ny]; when set they replace
    // vol and vol_t in the gathers
    const float4 *p4 = nullptr;
    const float4 *p4t = nullptr;
    // the same for a 16-bit volume: element (x, y, z) = the four 16-bit
    // corners in the order above, two to a 32-bit word, low half first
    const uint2 *p2 = nullptr;
    const uint2 *p2t = nullptr;
};

// Backprojection modes.
enum BpMode : int {
    BP_PLAIN = 0,     // vol += A^T sino
    BP_ONES = 1,      // vol += A^T 1 (sino ignored)
};

// Launchers (defined in the .hip translation units).  All asynchronous.
hipError_t launch_forward(const RayGrid &g, const WarpGrid &w, const void *vol, int vol_dtype,
                          void *out, int out_dtype, int mode, const FpExtra &ex,
                          hipStream_t stream);
// vol (+)= scale A^T sino; `Pmat` holds the view matrices [n_proj * n_sub][12]
// on the device.  accumulate == 0 overwrites vol.  `scratch` is one device
// float (max |sino|); `work` holds back_scratch_bytes(g, max_chunks, direct)
// bytes: the owner form's 64-bit integer volume, or the direct form's
// per-chunk partial volumes (may be null when that is 0).  The direct form
// (direct = true) needs no volume-sized buffer when one projection chunk
// suffices; max_chunks > 0 caps its chunks (0 = no cap).
hipError_t launch_back(const RayGrid &g, const WarpGrid &w, const double *Pmat, const void *sino,
                       int sino_dtype, float *vol, int accumulate, int mode, float *scratch,
                       void *work, hipStream_t stream, float scale = 1.0f, int max_chunks = 0,
                       bool direct = false);
size_t back_scratch_bytes(const RayGrid &g, int max_chunks = 0, bool direct = false);
// Where the voxel-driven backprojector's voxel centres sit: the Cartesian
// grid of the RayGrid (cyl == 0), or the polar grid of the cylindrical domain
// (cyl != 0: g.nx = n_r rings at (i + 1/2) dr, g.ny = n_phi angles 2 pi j /
// n_phi, g.nz = n_z slices (k - (n_z - 1)/2) dz, in the frame the matrices
// act on).
struct VoxelGrid {
    int cyl = 0;
    double dr = 1.0, dz = 1.0;
};

// vol (+)= B sino with the voxel-driven backprojector (ones != 0: B 1, sino
// ignored); deterministic, no scratch.  Needs n_u, n_v >= 2.
hipError_t launch_back_voxel(const RayGrid &g, const double *Pmat, const void *sino, int sino_dtype,
                             float *vol, int accumulate, int ones, const VoxelGrid &vg,
                             hipStream_t stream);

// The aligned cylindrical domain: polar grid [nz][nphi][nr] about the z axis
// of the cylinder frame; the RayGrid's table then holds every sub-view's
// source and R_p M^-1 in that frame.
struct CylGrid {
    int nr, nphi, nz;
    float inv_dr, inv_dz, half_z, phi_scale;  // 1/dr, 1/dz, (nz-1)/2, nphi/(2 pi)
    double rh2, hz;                           // hull radius^2 and half height
};
CylGrid make_cyl_grid(int nr, int nphi, int nz, double dr, double dz);
hipError_t launch_forward_cyl(const RayGrid &g, const CylGrid &c, const void *vol, int vol_dtype,
                              void *out, int out_dtype, int mode, const FpExtra &ex,
                              hipStream_t stream);
hipError_t launch_sample_count_cyl(const RayGrid &g, const CylGrid &c, unsigned long long *count,
                                   hipStream_t stream);
// *out = max |x_i| over n elements (out is overwritten).
hipError_t launch_max_abs(const void *x, int dtype, size_t n, float *out, hipStream_t stream);
hipError_t launch_sample_count(const RayGrid &g, unsigned long long *count, hipStream_t stream);
hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t stream);
hipError_t launch_recip(float *a, size_t n, hipStream_t stream);
// x <- x + alpha C w z (w optional voxel weights), clamp, 16-bit shadow
hipError_t launch_update(float *x, const float *z, const float *C, const float *w, float alpha,
                         int nonneg, void *shadow, int shadow_dtype, size_t n, hipStream_t stream);
// dst = src with x and y exchanged ([nz][ny][nx] -> [nz][nx][ny]); dtype
// gives the element size.
hipError_t launch_transpose_xy(const void *src, void *dst, int dtype, int nx, int ny, int nz,
                               hipStream_t s);
// p4 / p4t = the corner-packed copies of FpExtra (either may be null).
hipError_t launch_pack_corners(const float *vol, float4 *p4, float4 *p4t, int nx, int ny, int nz,
                               hipStream_t s);
// The same corner-packed copies of a 16-bit volume (BF16 or F16 bits).
hipError_t launch_pack_corners16(const uint16_t *vol, uint2 *p2, uint2 *p2t, int nx, int ny,
                                 int nz, hipStream_t s);
// Corner-packed copy of a polar volume [nz][nphi][nr]: element (k, j, a) holds
// v(a, j), v(a+1, j), v(a, j+1), v(a+1, j+1) of slice k, the angle periodic.
hipError_t launch_pack_polar(const float *vol, float4 *p4, int nr, int nphi, int nz,
                             hipStream_t s);
hipError_t launch_convert(const void *src, int src_dtype, void *dst, int dst_dtype, size_t n,
                          hipStream_t stream);
hipError_t launch_sum_partials(const double *partials, int n, double *out, hipStream_t stream);
hipError_t launch_repack_warp(const float *U, float4 *out, size_t n_nodes, hipStream_t stream);

// Total variation: per-block FP64 partial sums (tv_blocks(n) of them) and the
// weighted gradient.
int tv_blocks(size_t n);
hipError_t launch_tv_value(const float *x, int nx, int ny, int nz, float eps, double *partials,
                           hipStream_t s);
hipError_t launch_tv_grad(const float *x, int nx, int ny, int nz, float eps, float weight,
                          float *g, hipStream_t s);

// Detector tile processed by one workgroup of the projectors.
constexpr int TILE_U = 16;
constexpr int TILE_V = 16;
constexpr int PROJ_THREADS = TILE_U * TILE_V;
constexpr int N_XCD = 8;

}  // namespace ctrex
