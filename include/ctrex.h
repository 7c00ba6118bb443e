/*
 * ctrex.h — C ABI of the MI355X ray-driven projector library.
 *
 * The library evaluates the projection–correction–backprojection loop of the
 * CTrex paper (arxiv 2609.30166): the forward projector A (Sec. 4.1,
 * "Projection operator"), the detector-space correction R(p - A mu)
 * (Sec. 4.1, "Correction kernel"), the backprojector A^T with voxel
 * normalisation C (Sec. 4.1, "Backprojection operator") and the SIRT update of
 * Eq. (1) (Sec. 2.3.1), over per-projection 3x4 view matrices (Sec. 2.2), with
 * optional angular sub-samples (Sec. 3.4, 4.2.2) and a displacement-field warp
 * applied during ray traversal (Sec. 3.1, 4.2.1).
 *
 * Conventions (all entry points):
 *  - Volume frame V: voxel units, centred; voxel (ix, iy, iz) has its centre at
 *    (ix - (nx-1)/2, iy - (ny-1)/2, iz - (nz-1)/2).  Volumes are contiguous
 *    [nz][ny][nx] arrays (x fastest).
 *  - View matrices: float64, row-major [n_proj][n_sub][3][4]; P (X, 1)^T is
 *    proportional to (u, v, 1)^T with (u, v) in pixel-index units (pixel
 *    (iu, iv) centred at (iu, iv)).  Only the line through the source and the
 *    pixel centre matters, so P may carry any non-zero scale or sign.
 *  - Sinograms: contiguous [n_views][n_v][n_u] (u fastest); row k belongs to
 *    projection views[k] (or k when views == NULL).
 *  - The ray of pixel (iu, iv) is clipped to the voxel-centre hull
 *    [0, nx-1] x [0, ny-1] x [0, nz-1] (index coordinates), sampled at the
 *    midpoints of n = ceil(L / step) equal parts of its chord L, each sample
 *    interpolated trilinearly and weighted by its length L / n.  Sub-views
 *    are averaged.  A warped sample that leaves the hull contributes zero.
 *  - Device pointers are HIP device memory owned by the caller; host pointers
 *    are read during the call only.  `stream` is a hipStream_t (NULL = the
 *    null stream).  Launches are asynchronous on that stream unless stated.
 *  - Buffers: every volume- or sinogram-sized intermediate lives in memory the
 *    caller provides (Sec. 2.1: the reconstruction control prepares the
 *    volume buffers): the SIRT workspace argument, and the device scratch
 *    attached with ctrex_set_scratch and sized by ctrex_scratch_bytes.  The
 *    context itself keeps only its geometry table, the repacked motion grid,
 *    device copies of up to 64 recent view lists and a few reduction cells.
 *  - Every entry point returns CTREX_OK or a negative status; the message of
 *    the last failure on a context is returned by ctrex_last_error().
 *    Arguments are validated on the host before anything is launched; a
 *    failed call launches nothing.  A context is not thread-safe, and calls on
 *    one context must be ordered (one stream, or caller synchronisation).
 */
#ifndef CTREX_H
#define CTREX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define CTREX_API __attribute__((visibility("default")))
#else
#define CTREX_API
#endif

typedef struct ctrex_ctx ctrex_ctx;

/* Status codes. */
#define CTREX_OK 0
#define CTREX_EINVAL (-1)         /* bad argument (NULL pointer, bad enum, ...) */
#define CTREX_ESHAPE (-2)         /* sizes inconsistent or out of range */
#define CTREX_ESINGULAR (-3)      /* a view matrix's 3x3 block is singular */
#define CTREX_ESOURCE_INSIDE (-4) /* a source lies inside the volume hull */
#define CTREX_EDEVICE (-5)        /* HIP runtime error (including earlier faults) */
#define CTREX_EWORKSPACE (-6)     /* workspace missing or too small */
#define CTREX_ESTATE (-7)         /* call order: no geometry set, ... */
#define CTREX_ENONFINITE (-8)     /* a residual norm came out NaN or Inf */

/* Storage types of volumes and sinograms.  Arithmetic is always FP32 with FP32
 * accumulation; geometry (inversion, clipping) is FP64.  16-bit stores round
 * to nearest even. */
#define CTREX_F32 0
#define CTREX_BF16 1
#define CTREX_F16 2

/* Flags of ctrex_sirt_iterate. */
#define CTREX_NONNEG 1u        /* clamp the volume at zero after every update */
#define CTREX_BF16_GATHER 2u   /* ray-march a BF16 shadow of the FP32 volume */
#define CTREX_F16_GATHER 4u    /* ray-march an FP16 shadow of the FP32 volume */
#define CTREX_RECOMPUTE_WEIGHTS 8u /* rebuild R and C even if cached */
#define CTREX_VOXEL_BP 16u     /* backproject with ctrex_back_project_voxel's B */

/* Create a context bound to HIP device `device`. */
CTREX_API int ctrex_create(ctrex_ctx **out, int device);

/*
 * Device scratch the projector calls need (Sec. 2.1: buffers are prepared by
 * the reconstruction control, here the caller).  ctrex_scratch_bytes returns
 * the bytes the calls of the current geometry (and cylindrical domain, if
 * set) need for view lists of up to n_views entries (n_views <= 0: n_proj):
 * the correction volume (4 bytes per voxel), a 16-bit shadow (2), the
 * copies of the volume the rays gather from (32 for FP32, 16 for 16-bit;
 * the backprojector's 64-bit integer sums, 8 per voxel, reuse that region)
 * and the residual partials (8 per 16x16 detector tile per view).
 * CTREX_ESTATE without a geometry.
 * ctrex_set_scratch attaches `bytes` of device memory at `dev` (NULL, 0
 * detaches; `dev` 256-byte aligned, as hipMalloc returns it, CTREX_EINVAL
 * otherwise).  The library keeps the pointer: the memory must stay allocated
 * and must not be written by the caller while calls that use it may run.
 * Calls that need more scratch than is attached return CTREX_EWORKSPACE
 * before launching anything; the library never allocates it itself.  The
 * learned-correction calls of ctrex_nn.h use the same attachment.
 */
CTREX_API int ctrex_scratch_bytes(const ctrex_ctx *ctx, int32_t n_views, size_t *bytes);
CTREX_API int ctrex_set_scratch(ctrex_ctx *ctx, void *dev, size_t bytes);

/* Destroy a context (NULL is accepted).  Waits for the device first. */
CTREX_API void ctrex_destroy(ctrex_ctx *ctx);

/* Message of the last failed call on `ctx` (never NULL). */
CTREX_API const char *ctrex_last_error(const ctrex_ctx *ctx);

/*
 * Sec. 2.2 (single-projection geometry, trajectory representation): install
 * the per-projection geometry.  `view_matrices` is a host float64 array
 * [n_proj][n_sub][3][4].  For every sub-view the library computes, in FP64,
 * the inverse of the left 3x3 block M and the source S = -M^-1 P[:, 3]; it
 * rejects |det M| < 1e-12 ||M||_F^3 (CTREX_ESINGULAR) and sources inside
 * the hull (CTREX_ESOURCE_INSIDE).  Volume sides must be >= 2 and < 2^22
 * with nx*ny*nz < 2^31; step > 0 with fewer than 2^24 steps along the hull
 * diagonal.  The table is copied to the device
 * synchronously.  Clears any motion field and invalidates cached SIRT weights.
 */
CTREX_API int ctrex_set_geometry(ctrex_ctx *ctx, const double *view_matrices, int32_t n_proj,
                       int32_t n_sub, int32_t n_u, int32_t n_v, int32_t nx, int32_t ny,
                       int32_t nz, double step);

/*
 * Sec. 3.1 / 4.2.1 (displacement field applied during ray traversal): every
 * sample c of sub-view (p, s) is moved to c + tau[p][s] * U(c) before the
 * lookup, U interpolated trilinearly from a device float32 grid
 * `U_dev` [gz][gy][gx][3] (x, y, z components, voxel units) whose nodes span
 * the hull (node k of an axis at index coordinate k (n-1)/(g-1)); lookups
 * clamp to the grid.  `tau` is a host float64 [n_proj][n_sub] array.  The grid
 * is copied (repacked) by the library; U_dev may be freed after the call,
 * which synchronises the device.  U_dev == NULL removes the warp.  Grid sides
 * must be >= 2.  Invalidates cached SIRT weights.
 */
CTREX_API int ctrex_set_motion(ctrex_ctx *ctx, const float *U_dev, int32_t gx, int32_t gy, int32_t gz,
                     const double *tau);

/*
 * Weighted backprojection (Sec. 3.2, 4.3.2): voxel weights w_j in [0, 1]
 * scale the correction each voxel accumulates in ctrex_sirt_iterate, so the
 * update becomes vol <- vol + alpha C w (A^T R (sino - A vol)); regions of
 * weight 0 keep their starting values (a reference volume passed as `vol`).
 * Since w_j is constant per voxel this equals weighting every contribution
 * inside the backprojection's accumulation.  `w_dev`: device FP32 array of
 * nx*ny*nz weights in the volume layout, owned by the caller and kept alive
 * while set (the library stores the pointer); NULL removes the weights.
 * ctrex_back_project itself stays the exact transpose.  Needs a geometry;
 * ctrex_set_geometry removes the weights.
 */
CTREX_API int ctrex_set_voxel_weights(ctrex_ctx *ctx, const float *w_dev);

/*
 * Sec. 4.1 (projection operator): sino = A vol for the projections in
 * `views` (host int32 list of n_views indices in [0, n_proj), repeats
 * allowed; NULL selects all projections in order).  `vol` has storage type
 * vol_dtype and `sino` sino_dtype; the sinogram is overwritten.  With an
 * empty list (n_views == 0) nothing happens and the pointers may be NULL.
 * The rays gather from copies of `vol` written into the attached scratch at
 * the start of the call: two corner-packed copies (x- and y-fastest; each
 * element holds a voxel's four corner values in its z slice: 16 bytes for
 * float32, 8 bytes for 16-bit storage).  The results do not depend on which
 * copy a ray reads.
 */
CTREX_API int ctrex_forward_project(ctrex_ctx *ctx, const void *vol, int32_t vol_dtype, void *sino,
                          int32_t sino_dtype, const int32_t *views, int32_t n_views,
                          void *stream);

/*
 * Sec. 4.1 (backprojection operator), as the exact transpose of
 * ctrex_forward_project: vol (+)= A^T sino over the listed projections.
 * `vol` is a device float32 volume; with accumulate == 0 it is zeroed first
 * (also for an empty view list, where `sino` may be NULL).
 * Contributions are summed as 64-bit fixed-point integers (scale chosen from
 * max |sino| so no sum overflows), so the result is bitwise reproducible
 * from run to run.  A context cell holds max |sino|; the integer sums are
 * kept in the attached scratch (8 bytes per voxel, in the region of the
 * forward projector's gather copies) and scaled into `vol` at the end.
 */
CTREX_API int ctrex_back_project(ctrex_ctx *ctx, const void *sino, int32_t sino_dtype, float *vol,
                       int32_t accumulate, const int32_t *views, int32_t n_views,
                       void *stream);

/*
 * vol (+)= scale A^T sino: ctrex_back_project with every contribution
 * multiplied by the finite factor `scale` (inside the fixed-point sums, so
 * no extra pass over the volume).  The gradient of the data term of Eq. (1),
 * 2 A^T (A x - b), is ctrex_data_residual's r backprojected with scale 2.
 */
CTREX_API int ctrex_back_project_scaled(ctrex_ctx *ctx, const void *sino, int32_t sino_dtype,
                                        float scale, float *vol, int32_t accumulate,
                                        const int32_t *views, int32_t n_views, void *stream);

/*
 * ctrex_back_project without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same operator, arguments, layouts and
 * errors as ctrex_back_project; it never calls hipMalloc or hipFree and
 * needs no attached scratch.  Its scratch is a fixed 32 MiB array of the
 * library on each GPU (held until the process ends): the view list (at most
 * 262144 entries, else CTREX_ESHAPE before any launch), the max |sino|
 * cell, and the per-chunk partial volumes, whose number is capped to what
 * fits (one chunk, and no partial volume, when even two do not), so large
 * volumes differ from ctrex_back_project only by the rounding of the
 * fixed-point scale.  With a view list the call waits for `stream` (the
 * list is copied into the array).  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads or
 * contexts) race and must be serialised by the caller.
 */
CTREX_API int ctrex_back_project_noalloc(ctrex_ctx *ctx, const void *sino, int32_t sino_dtype,
                                         float *vol, int32_t accumulate, const int32_t *views,
                                         int32_t n_views, void *stream);

/*
 * Sec. 4.1 (backprojection operator), the paper's voxel-driven form:
 * vol (+)= B sino over the listed projections, where for voxel j with centre
 * X_j (V frame, index coordinates centred on the volume) and each sub-view
 * (p, s) the detector point (u, v), P_{p,s} (X_j, 1)^T ~ (u, v, 1)^T, samples
 * the image of projection p bilinearly (pixel centres at integer u, v; zero
 * beyond the border):  z_j = (1 / n_sub) sum_{p, s} r_p(u, v).  A view whose
 * depth row vanishes at X_j (the voxel lies in the source's detector-parallel
 * plane) contributes nothing.  B is not the transpose of
 * ctrex_forward_project; ctrex_sirt_iterate pairs it with C = 1 / (B 1) under
 * CTREX_VOXEL_BP.  Arguments, layouts and the empty list behave as in
 * ctrex_back_project.  Each voxel is summed by one thread in FP64 in view
 * order, so results are deterministic.  Needs 2 <= n_u, n_v < 2^24 and
 * n_u n_v < 2^30 (CTREX_ESHAPE) and no motion field (CTREX_ESTATE).
 */
CTREX_API int ctrex_back_project_voxel(ctrex_ctx *ctx, const void *sino, int32_t sino_dtype,
                                       float *vol, int32_t accumulate, const int32_t *views,
                                       int32_t n_views, void *stream);

/*
 * Bytes of device workspace ctrex_sirt_iterate needs for n_views projections
 * (n_views <= 0 means all): R and the correction image (one value per ray
 * each), C (one value per voxel) and per-tile residual partials.  `flags` is
 * accepted for compatibility and does not change the size.
 */
CTREX_API int ctrex_sirt_workspace_bytes(const ctrex_ctx *ctx, int32_t n_views, uint32_t flags,
                               size_t *bytes);

/*
 * Eq. (1) with the listed projections as the subset P_k (Sec. 2.3.1, 2.3.2):
 *   vol <- vol + alpha C A^T R (sino - A vol), repeated n_iter times,
 * with R = 1 / (A 1) and C = 1 / (A^T 1) (zero where a sum is zero); with
 * CTREX_VOXEL_BP the voxel-driven B of ctrex_back_project_voxel takes the
 * place of A^T, and C = 1 / (B 1).
 * `vol` is the device float32 volume (in/out); `sino` the measured data
 * (device, sino_dtype, [n_views][n_v][n_u]).  `workspace` is caller-owned
 * device memory of at least ctrex_sirt_workspace_bytes(); it holds R, C, the
 * correction image and residual partials, and R and C are kept there between
 * calls for the same
 * geometry, motion, view list and workspace (CTREX_RECOMPUTE_WEIGHTS forces
 * a rebuild; the caller must not write the workspace in between, and must
 * pass the flag after reusing freed memory at the same address as a
 * workspace).  The context remembers up to 64 (workspace, view list) pairs,
 * so ordered subsets — one workspace per subset, cycled — keep their
 * weights.  The volume-sized intermediates (the correction volume, a 16-bit
 * shadow and the copies of vol the rays gather from: 32 bytes per voxel in
 * FP32, 16 with a 16-bit gather) live in the attached scratch, shared by all
 * workspaces.  With a
 * BF16/F16 gather flag the rays march a 16-bit shadow of vol, refreshed
 * after every update, while the update itself stays FP32.  The correction
 * image R (sino - A vol) is stored in sino_dtype.  If `resid_norms` (host,
 * n_iter doubles) is non-NULL the call waits for the stream and stores
 * ||sino - A vol_k||_2 of every iterate k = 0..n_iter-1 (k = 0 is the input
 * volume) and returns CTREX_ENONFINITE if any is NaN or Inf; otherwise it
 * returns without waiting.
 */
CTREX_API int ctrex_sirt_iterate(ctrex_ctx *ctx, float *vol, const void *sino, int32_t sino_dtype,
                       int32_t n_iter, float alpha, uint32_t flags, const int32_t *views,
                       int32_t n_views, void *workspace, size_t workspace_bytes,
                       double *resid_norms, void *stream);

/*
 * Residual norm ||b - A vol||_2 of a volume against a measured sinogram over
 * the listed projections: the data-consistency measure of the SIRT update
 * (Eq. 1) and the acceptance test of a learned correction between
 * iterations (Sec. 5 extension).  `vol` and `sino` are device arrays laid
 * out as in ctrex_forward_project; the gather copies and per-tile partials
 * go to the attached scratch, and the projection is not stored.  Residuals
 * are formed in FP32 per detector pixel and squared and summed in FP64 in a
 * fixed order (deterministic).  Writes *norm (host) and waits for `stream`;
 * CTREX_ENONFINITE if the norm is not finite.
 */
CTREX_API int ctrex_residual_norm(ctrex_ctx *ctx, const void *vol, int32_t vol_dtype,
                                  const void *sino, int32_t sino_dtype, const int32_t *views,
                                  int32_t n_views, double *norm, void *stream);

/*
 * Data term of Eq. (1) for the differentiable loss ||A vol - b||^2 (the
 * residual b - A mu of the correction kernel, Sec. 4.1, with the opposite
 * sign): over the listed projections, r = scale (A vol - b) is stored in
 * `r` (device, sino_dtype, [n_views][n_v][n_u]; NULL: not stored) and
 * sum (A vol - b)^2 in `sq_sum` (one device float64; NULL: not computed).
 * Residuals are formed in FP32 per pixel; their squares are summed in FP64
 * in a fixed order (deterministic).  `b` has sino_dtype.  Asynchronous (no
 * host wait).  An empty view list zeroes *sq_sum and stores nothing.  The
 * gather copies and partials use the attached scratch, as in
 * ctrex_residual_norm.  At least one of r and sq_sum must be non-NULL.
 */
CTREX_API int ctrex_data_residual(ctrex_ctx *ctx, const void *vol, int32_t vol_dtype,
                                  const void *b, void *r, int32_t sino_dtype, float scale,
                                  const int32_t *views, int32_t n_views, double *sq_sum,
                                  void *stream);

/*
 * Exact number of ray samples (trilinear lookups) one forward projection of
 * the listed projections performs, summed over sub-views; synchronous.
 */
CTREX_API int ctrex_sample_count(ctrex_ctx *ctx, const int32_t *views, int32_t n_views, int64_t *count,
                       void *stream);

/*
 * Storage conversion of n elements between CTREX_F32/BF16/F16 device arrays
 * (round to nearest even), for callers preparing 16-bit inputs.
 */
CTREX_API int ctrex_convert(ctrex_ctx *ctx, const void *src, int32_t src_dtype, void *dst,
                  int32_t dst_dtype, int64_t n, void *stream);

/*
 * Total-variation regulariser for the differentiable loss
 * ||A x - b||^2 + weight * TV(x) (an extension: the paper's Sec. 5 names
 * regularisers among the learned or hybrid components its operators admit).
 * TV(x) = sum_j sqrt(|D x_j|^2 + eps^2), D the forward differences along x, y
 * and z with a zero difference at the last index of each axis.  `x` is a
 * device float32 [nz][ny][nx] volume (any geometry; none needs to be set).
 * If `value` (host) is non-NULL the call waits for the stream and stores
 * TV(x), summed in FP64 in a fixed order.  If `grad` (device float32, same
 * shape, not aliasing x) is non-NULL it is overwritten with weight * dTV/dx.
 */
CTREX_API int ctrex_tv(ctrex_ctx *ctx, const float *x, int32_t nx, int32_t ny, int32_t nz,
                       float eps, float weight, double *value, float *grad, void *stream);

/*
 * Kernel timing of ctrex_sirt_iterate (instrumentation, no effect on
 * results).  With profiling enabled, every iteration records HIP events on
 * the launch stream around its forward-projection-with-correction, its
 * backprojection and its update launches.  ctrex_profile_read waits for the
 * device, returns the summed milliseconds and launch counts of the three
 * phases (ms[3], launches[3]: forward, back, update) since the last read,
 * and clears them.  Enabling clears earlier records.
 */
CTREX_API int ctrex_profile_enable(ctrex_ctx *ctx, int32_t enable);
CTREX_API int ctrex_profile_read(ctrex_ctx *ctx, double *ms, int64_t *launches);

/*
 * Aligned cylindrical volume domain (Sec. 3.5; the projector's and the
 * backprojector's geometry-level modifications, Sec. 4.2.1 and 4.3.1).
 *
 * The volume is a polar grid about the z axis of a cylinder frame, stored
 * [n_z][n_phi][n_r] float (r fastest): ring i at radius (i + 1/2) dr, angle
 * j at 2 pi j / n_phi (periodic), slice k at (k - (n_z - 1)/2) dz.  `pose`
 * (host float64 [3][4] = [R | t], or NULL for the identity) is the rigid map
 * X_c = R X + t from the V frame of the view matrices to the cylinder frame;
 * R must be a rotation (|R^T R - I| <= 1e-9, det +1) or CTREX_EINVAL.
 * The projector clips each ray of ctrex_forward_project to the hull
 * r <= (n_r - 1/2) dr, |z| <= (n_z - 1) dz / 2 (not the box), samples it at
 * the midpoints of n = ceil(L / step) equal parts (weight L / n each) and
 * looks up the grid trilinearly in (r / dr - 1/2, phi n_phi / (2 pi),
 * z / dz + (n_z - 1)/2), the radial index clamped to [0, n_r - 1] (the core
 * r < dr/2 takes the innermost ring's values) and the angle periodic; sub-views
 * are averaged.  The backprojector is the voxel-driven one of
 * ctrex_back_project_voxel over the polar voxel centres.  ctrex_set_cylinder
 * needs a geometry (its view matrices and step; the box sides of
 * ctrex_set_geometry play no part here), computes every sub-view's source and
 * ray map in the cylinder frame, and rejects sources inside the cylinder
 * (CTREX_ESOURCE_INSIDE); n_r >= 2, n_phi >= 3, n_z >= 2, fewer than 2^31
 * voxels (CTREX_ESHAPE); dr, dz > 0.  ctrex_set_geometry removes the
 * cylinder.  The cylinder calls return CTREX_ESTATE without a cylinder or
 * with a motion field set (no warp on this domain).
 */
CTREX_API int ctrex_set_cylinder(ctrex_ctx *ctx, int32_t n_r, int32_t n_phi, int32_t n_z,
                                 double dr, double dz, const double *pose);

/* sino = A_cyl vol over the listed projections (arguments as in
 * ctrex_forward_project; `vol` is the polar grid). */
CTREX_API int ctrex_forward_project_cyl(ctrex_ctx *ctx, const void *vol, int32_t vol_dtype,
                                        void *sino, int32_t sino_dtype, const int32_t *views,
                                        int32_t n_views, void *stream);

/* vol (+)= B_cyl sino: the voxel-driven backprojector over the polar voxel
 * centres (mapped to the V frame; arguments, determinism and detector limits
 * as in ctrex_back_project_voxel). */
CTREX_API int ctrex_back_project_cyl(ctrex_ctx *ctx, const void *sino, int32_t sino_dtype,
                                     float *vol, int32_t accumulate, const int32_t *views,
                                     int32_t n_views, void *stream);

/* Exact number of samples of one cylindrical forward projection; synchronous. */
CTREX_API int ctrex_sample_count_cyl(ctrex_ctx *ctx, const int32_t *views, int32_t n_views,
                                     int64_t *count, void *stream);

/* Workspace bytes of ctrex_sirt_iterate_cyl for n_views projections (<= 0: all). */
CTREX_API int ctrex_sirt_workspace_bytes_cyl(const ctrex_ctx *ctx, int32_t n_views,
                                             size_t *bytes);

/*
 * Eq. (1) on the cylindrical domain: vol <- vol + alpha C B R (sino - A vol)
 * with A, B the cylinder operators above, R = 1 / (A 1), C = 1 / (B 1).
 * Arguments, the workspace and its weight cache, the attached scratch (here
 * the correction volume and the packed copy of vol, 20 bytes per voxel) and
 * the residual norms as in ctrex_sirt_iterate; flags CTREX_NONNEG and
 * CTREX_RECOMPUTE_WEIGHTS only (the volume is FP32; no voxel weights).
 */
CTREX_API int ctrex_sirt_iterate_cyl(ctrex_ctx *ctx, float *vol, const void *sino,
                                     int32_t sino_dtype, int32_t n_iter, float alpha,
                                     uint32_t flags, const int32_t *views, int32_t n_views,
                                     void *workspace, size_t workspace_bytes,
                                     double *resid_norms, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CTREX_H */
