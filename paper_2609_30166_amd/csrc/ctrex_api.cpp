// Host runtime of libctrex: the C ABI declared in include/ctrex.h.
//
// Owns the per-context device geometry table (FP64 source + inverse matrix
// per sub-view), the repacked motion grid, device copies of view lists and a
// few fixed-size reduction cells; every volume- or sinogram-sized buffer is
// the caller's (the workspace of the SIRT calls and the scratch attached with
// ctrex_set_scratch).  Validation happens before any launch, so a failing call
// leaves the device untouched.

#include "../../include/ctrex.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "ctrex_ctx.h"
#include "ctrex_internal.h"

using namespace ctrex;

namespace {

constexpr size_t kAlign = 256;
constexpr int kResidCap = 1024;
constexpr size_t kMaxLists = 64;
constexpr size_t kMaxWeightSets = 64;
// FP32 volumes are gathered from corner-packed copies (two 16-byte loads per
// sample instead of four 8-byte ones); 16-bit volumes from the plain copies.
constexpr bool kPackedCorners = true;
// The same for 16-bit volumes: two corner-packed copies of 8 bytes per voxel.
constexpr bool kPacked16 = true;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool valid_dtype(int32_t t) { return t == CTREX_F32 || t == CTREX_BF16 || t == CTREX_F16; }
size_t dtype_size(int32_t t) { return t == CTREX_F32 ? 4 : 2; }

// Inverse of a 3x3 matrix through cyclic cofactors; returns the determinant.
double invert3(const double m[3][3], double inv[3][3]) {
    double cof[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            cof[i][j] = m[i1][j1] * m[i2][j2] - m[i1][j2] * m[i2][j1];
        }
    const double det = m[0][0] * cof[0][0] + m[0][1] * cof[0][1] + m[0][2] * cof[0][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) inv[j][i] = cof[i][j] / det;
    return det;
}

// Select (and upload once) the device copy of a view list.  NULL = all views.
int resolve_views(ctrex_ctx *c, const int32_t *views, int32_t n_views, const int32_t **dev,
                  int32_t *count, hipStream_t stream) {
    if (!views) {
        *dev = nullptr;
        *count = c->n_proj;
        return CTREX_OK;
    }
    if (n_views < 0) return fail(c, CTREX_ESHAPE, "n_views must be >= 0 (got %d)", n_views);
    for (int32_t k = 0; k < n_views; ++k)
        if (views[k] < 0 || views[k] >= c->n_proj)
            return fail(c, CTREX_ESHAPE, "views[%d] = %d outside [0, %d)", k, views[k], c->n_proj);
    *count = n_views;
    if (n_views == 0) {
        *dev = nullptr;
        return CTREX_OK;
    }
    for (auto it = c->lists.begin(); it != c->lists.end(); ++it) {
        if (static_cast<int32_t>(it->host.size()) == n_views &&
            std::memcmp(it->host.data(), views, sizeof(int32_t) * n_views) == 0) {
            c->lists.splice(c->lists.begin(), c->lists, it);
            *dev = c->lists.front().dev;
            return CTREX_OK;
        }
    }
    DeviceViewList l;
    l.host.assign(views, views + n_views);
    CTREX_HIP(c, hipMalloc(&l.dev, sizeof(int32_t) * n_views));
    hipError_t e = hipMemcpyAsync(l.dev, l.host.data(), sizeof(int32_t) * n_views,
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        (void)hipFree(l.dev);
        return hip_fail(c, e, "upload of view list");
    }
    c->lists.push_front(std::move(l));
    while (c->lists.size() > kMaxLists) {
        // the evicted list's last use was ordered before this synchronised upload
        (void)hipFree(c->lists.back().dev);
        c->lists.pop_back();
    }
    *dev = c->lists.front().dev;
    return CTREX_OK;
}

}  // namespace

int ctrex::ctx_scratch(ctrex_ctx *c, size_t bytes, void **out) {
    *out = c->user_scratch;
    if (bytes == 0) return CTREX_OK;
    if (!c->user_scratch || c->user_scratch_bytes < bytes)
        return fail(c, CTREX_EWORKSPACE,
                    "this call needs %zu bytes of device scratch, %zu attached "
                    "(ctrex_set_scratch; size from ctrex_scratch_bytes)",
                    bytes, c->user_scratch_bytes);
    return CTREX_OK;
}

namespace {

RayGrid make_grid(const ctrex_ctx *c, const int32_t *dev_views, int32_t n_views) {
    RayGrid g;
    g.tab = c->d_tab;
    g.views = dev_views;
    g.n_views = n_views;
    g.n_sub = c->n_sub;
    g.n_u = c->n_u;
    g.n_v = c->n_v;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.step = c->step;
    g.tiles_u = (c->n_u + TILE_U - 1) / TILE_U;
    g.tiles_v = (c->n_v + TILE_V - 1) / TILE_V;
    const long long total = static_cast<long long>(g.tiles_u) * g.tiles_v * n_views;
    g.total_blocks = static_cast<int>(total);
    g.tube = c->fp_tube;
    return g;
}

WarpGrid make_warp(const ctrex_ctx *c) {
    WarpGrid w;
    w.U = c->d_U;
    w.gx = c->gx;
    w.gy = c->gy;
    w.gz = c->gz;
    w.sx = c->d_U ? double(c->gx - 1) / double(c->nx - 1) : 0.0;
    w.sy = c->d_U ? double(c->gy - 1) / double(c->ny - 1) : 0.0;
    w.sz = c->d_U ? double(c->gz - 1) / double(c->nz - 1) : 0.0;
    w.fsx = static_cast<float>(w.sx);
    w.fsy = static_cast<float>(w.sy);
    w.fsz = static_cast<float>(w.sz);
    w.margin = c->d_U ? c->warp_margin : 0;
    w.umax = c->d_U ? c->warp_umax : 0.0;
    return w;
}

int check_ready(ctrex_ctx *c) {
    if (!c) return CTREX_EINVAL;
    if (!c->have_geom) return fail(c, CTREX_ESTATE, "no geometry set (call ctrex_set_geometry)");
    CTREX_HIP(c, hipSetDevice(c->device));
    return CTREX_OK;
}

int check_blocks(ctrex_ctx *c, int32_t n_views) {
    const long long tiles = static_cast<long long>((c->n_u + TILE_U - 1) / TILE_U) *
                            ((c->n_v + TILE_V - 1) / TILE_V);
    if (tiles * n_views > (1ll << 30))
        return fail(c, CTREX_ESHAPE, "too many detector tiles in one call (%lld)", tiles * n_views);
    const long long pix = static_cast<long long>(c->n_u) * c->n_v * n_views;
    if (pix >= (1ll << 31))
        return fail(c, CTREX_ESHAPE, "sinogram of %lld pixels exceeds 2^31 - 1", pix);
    return CTREX_OK;
}

hipError_t take_event(ctrex_ctx *c, hipEvent_t *e) {
    if (!c->ev_pool.empty()) {
        *e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Record an event pair around `phase` when profiling (start = true opens it).
struct PhaseTimer {
    ctrex_ctx *c;
    hipStream_t s;
    hipEvent_t a = nullptr;
    int phase;
    hipError_t begin() {
        if (!c->profiling) return hipSuccess;
        hipError_t e = take_event(c, &a);
        if (e != hipSuccess) return e;
        return hipEventRecord(a, s);
    }
    hipError_t end() {
        if (!c->profiling) return hipSuccess;
        hipEvent_t b;
        hipError_t e = take_event(c, &b);
        if (e != hipSuccess) return e;
        e = hipEventRecord(b, s);
        c->ev_marks.push_back({phase, {a, b}});
        return e;
    }
};

// The caller's workspace holds what a (workspace, view list) pair keeps:
// R, the correction image r, C and the residual partials.  The per-call
// volume-sized intermediates (the correction volume z, a 16-bit shadow and
// the copies the rays gather from) live in the scratch the caller attaches
// (ctrex_set_scratch), which all workspaces share, so ordered subsets cost
// one volume (C) per subset.
struct SirtLayout {
    size_t R, r, C, partials, resid, total;
};

// The caller's scratch (ctrex_set_scratch), as the Cartesian projector calls
// use it: the correction volume z, a 16-bit shadow, one region shared by the
// gather copies of the forward projector (FP32: two corner-packed copies of
// 16 bytes per voxel; 16-bit: 8 bytes each) and the backprojector's
// per-chunk partial volumes (never live at the same time), and the residual
// partials.  Each call needs the prefix up to the last region it uses.
struct ProjScratch {
    size_t z, shadow, shared, partials, total;
};

SirtLayout sirt_layout(const ctrex_ctx *c, int32_t n_views) {
    const size_t rays = static_cast<size_t>(n_views) * c->n_u * c->n_v;
    const size_t vox = static_cast<size_t>(c->nx) * c->ny * c->nz;
    const size_t tiles = static_cast<size_t>((c->n_u + TILE_U - 1) / TILE_U) *
                         ((c->n_v + TILE_V - 1) / TILE_V) * n_views;
    SirtLayout l;
    size_t off = 0;
    l.R = off;
    off = align_up(off + 4 * rays);
    l.r = off;
    off = align_up(off + 4 * rays);
    l.C = off;
    off = align_up(off + 4 * vox);
    l.partials = off;
    off = align_up(off + 8 * tiles);
    l.resid = off;
    off = align_up(off + 8 * kResidCap);
    l.total = off;
    return l;
}

size_t packed_bytes(const ctrex_ctx *c, int vol_dtype) {
    const size_t vox = static_cast<size_t>(c->nx) * c->ny * c->nz;
    if (vol_dtype == F32) return kPackedCorners ? 2 * sizeof(float4) * vox : 4 * vox;
    return kPacked16 ? 2 * sizeof(uint2) * vox : 2 * vox;
}

ProjScratch proj_scratch(const ctrex_ctx *c, int32_t n_views) {
    const size_t vox = static_cast<size_t>(c->nx) * c->ny * c->nz;
    const size_t tiles = static_cast<size_t>((c->n_u + TILE_U - 1) / TILE_U) *
                         ((c->n_v + TILE_V - 1) / TILE_V) * static_cast<size_t>(n_views);
    const size_t bpw = n_views > 0 ? back_scratch_bytes(make_grid(c, nullptr, n_views)) : 0;
    ProjScratch l;
    size_t off = 0;
    l.z = off;
    off = align_up(off + 4 * vox);
    l.shadow = off;
    off = align_up(off + 2 * vox);
    l.shared = off;
    off = align_up(off + std::max(packed_bytes(c, F32), bpw));
    l.partials = off;
    off = align_up(off + 8 * (tiles + 1));
    l.total = off;
    return l;
}

// The cylindrical domain's calls: the correction volume, then the
// corner-packed copy of the polar volume (16 bytes per voxel).
struct CylScratch {
    size_t z, packed, total;
};

// Write the copies of `vol` the rays gather from into `dst` (the shared
// region of the scratch) and point `ex` at them.
int make_gather_copies(ctrex_ctx *c, const void *vol, int vol_dtype, void *dst, FpExtra &ex,
                       hipStream_t s) {
    const size_t vox = static_cast<size_t>(c->nx) * c->ny * c->nz;
    if (kPackedCorners && vol_dtype == F32) {
        // corner-packed copies, x- and y-fastest
        float4 *p4 = static_cast<float4 *>(dst);
        CTREX_HIP(c, launch_pack_corners(static_cast<const float *>(vol), p4, p4 + vox, c->nx,
                                         c->ny, c->nz, s));
        ex.p4 = p4;
        ex.p4t = p4 + vox;
    } else if (kPacked16 && vol_dtype != F32) {
        // 16-bit corner-packed copies, x- and y-fastest
        uint2 *p2 = static_cast<uint2 *>(dst);
        CTREX_HIP(c, launch_pack_corners16(static_cast<const uint16_t *>(vol), p2, p2 + vox,
                                           c->nx, c->ny, c->nz, s));
        ex.p2 = p2;
        ex.p2t = p2 + vox;
    } else {
        // y-fastest copy for the projections whose rays run mainly along x
        CTREX_HIP(c, launch_transpose_xy(vol, dst, vol_dtype, c->nx, c->ny, c->nz, s));
        ex.vol_t = dst;
    }
    return CTREX_OK;
}

CylScratch cyl_scratch(const ctrex_ctx *c) {
    const size_t vox = static_cast<size_t>(c->cyl_nr) * c->cyl_nphi * c->cyl_nz;
    CylScratch l;
    l.z = 0;
    l.packed = align_up(4 * vox);
    l.total = align_up(l.packed + (kPackedCorners ? sizeof(float4) * vox : 0));
    return l;
}

// ---------------------------------------------- allocation-free backprojection --
// ctrex_back_project_noalloc keeps its scratch (the view list, the max |r|
// cell and the per-chunk partial volumes) in the fixed array below instead
// of the caller's or the library's allocations: one copy per GPU, held until
// the process ends.  In host code `scratch` names a host-side stand-in, not a
// device address; kernels are given the address hipGetSymbolAddress returns
// for the current device (kept in noalloc_ptr).
constexpr size_t kNoAllocBytes = size_t(32) << 20;
constexpr size_t kNoAllocViewBytes = size_t(1) << 20;   // up to 262144 projection indices
constexpr size_t kNoAllocMaxAbs = kNoAllocViewBytes;    // one float, its own 256-byte line
constexpr size_t kNoAllocSlabs = kNoAllocViewBytes + 256;
constexpr int kNoAllocDevices = 64;

std::mutex noalloc_mu;
void *noalloc_ptr[kNoAllocDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// Look up (once per device, with that device current) the device address of
// this GPU's copy of `scratch`.
int noalloc_setup(ctrex_ctx *c) {
    if (c->device < 0 || c->device >= kNoAllocDevices)
        return fail(c, CTREX_EDEVICE, "device %d beyond the %d the library supports", c->device,
                    kNoAllocDevices);
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (noalloc_ptr[c->device]) return CTREX_OK;
    CTREX_HIP(c, hipSetDevice(c->device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(c, CTREX_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    noalloc_ptr[c->device] = p;
    return CTREX_OK;
}

}  // namespace

extern "C" {

int ctrex_create(ctrex_ctx **out, int device) {
    if (!out) return CTREX_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return CTREX_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return CTREX_EDEVICE;
    ctrex_ctx *c = new ctrex_ctx();
    c->device = device;
    const char *gather = std::getenv("CTREX_FP_GATHER");
    c->fp_tube = gather && std::strcmp(gather, "lds") == 0;
    if (hipMalloc(&c->d_count, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->d_scalar, 4 * sizeof(float)) != hipSuccess ||
        hipMalloc(&c->d_red, sizeof(double) * 8193) != hipSuccess) {
        if (c->d_count) (void)hipFree(c->d_count);
        if (c->d_scalar) (void)hipFree(c->d_scalar);
        delete c;
        return CTREX_EDEVICE;
    }
    if (noalloc_setup(c) != CTREX_OK) {
        (void)hipFree(c->d_count);
        (void)hipFree(c->d_scalar);
        (void)hipFree(c->d_red);
        delete c;
        return CTREX_EDEVICE;
    }
    *out = c;
    return CTREX_OK;
}

void ctrex_destroy(ctrex_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &m : c->ev_marks) {
        c->ev_pool.push_back(m.second.first);
        c->ev_pool.push_back(m.second.second);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->d_tab) (void)hipFree(c->d_tab);
    if (c->d_P) (void)hipFree(c->d_P);
    if (c->d_tab_cyl) (void)hipFree(c->d_tab_cyl);
    if (c->d_P_cyl) (void)hipFree(c->d_P_cyl);
    if (c->d_U) (void)hipFree(c->d_U);
    if (c->d_count) (void)hipFree(c->d_count);
    if (c->d_scalar) (void)hipFree(c->d_scalar);
    if (c->d_red) (void)hipFree(c->d_red);
    for (auto &l : c->lists) (void)hipFree(l.dev);
    delete c;
}

const char *ctrex_last_error(const ctrex_ctx *c) {
    if (!c) return "null context";
    return c->err.c_str();
}

int ctrex_set_geometry(ctrex_ctx *c, const double *P, int32_t n_proj, int32_t n_sub, int32_t n_u,
                       int32_t n_v, int32_t nx, int32_t ny, int32_t nz, double step) {
    if (!c) return CTREX_EINVAL;
    if (!P) return fail(c, CTREX_EINVAL, "view_matrices is NULL");
    if (n_proj < 1 || n_sub < 1 || n_u < 1 || n_v < 1)
        return fail(c, CTREX_ESHAPE, "n_proj, n_sub, n_u, n_v must be >= 1");
    if (nx < 2 || ny < 2 || nz < 2) return fail(c, CTREX_ESHAPE, "volume sides must be >= 2");
    if (nx >= (1 << 22) || ny >= (1 << 22) || nz >= (1 << 22))
        return fail(c, CTREX_ESHAPE, "volume sides must be < 2^22");
    if (static_cast<long long>(nx) * ny * nz >= (1ll << 31))
        return fail(c, CTREX_ESHAPE, "volume of %lld voxels exceeds 2^31 - 1",
                    static_cast<long long>(nx) * ny * nz);
    if (static_cast<long long>(n_proj) * n_sub > (1 << 24))
        return fail(c, CTREX_ESHAPE, "too many sub-views");
    if (!(step > 0.0) || !std::isfinite(step)) return fail(c, CTREX_EINVAL, "step must be > 0");
    {
        // the longest chord (the hull diagonal) must need fewer than 2^24 samples,
        // so sample offsets stay exact in FP32 and every ray loop is short
        const double diag = std::sqrt(double(nx - 1) * (nx - 1) + double(ny - 1) * (ny - 1) +
                                      double(nz - 1) * (nz - 1));
        if (diag / step >= double(1 << 24))
            return fail(c, CTREX_EINVAL, "step %g too small for a hull diagonal of %g", step, diag);
    }
    CTREX_HIP(c, hipSetDevice(c->device));
    const size_t m = static_cast<size_t>(n_proj) * n_sub;
    std::vector<SubView> tab(m);
    const double half[3] = {0.5 * (nx - 1), 0.5 * (ny - 1), 0.5 * (nz - 1)};
    for (size_t k = 0; k < m; ++k) {
        const double *p = P + 12 * k;
        double M[3][3], Mi[3][3];
        double fro = 0.0;
        bool finite = true;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                M[i][j] = p[4 * i + j];
                fro += M[i][j] * M[i][j];
            }
        for (int i = 0; i < 12; ++i) finite = finite && std::isfinite(p[i]);
        if (!finite) return fail(c, CTREX_EINVAL, "view matrix %zu is not finite", k);
        fro = std::sqrt(fro);
        const double det = invert3(M, Mi);
        if (!(fro > 0.0) || !(std::fabs(det) >= 1e-12 * fro * fro * fro))
            return fail(c, CTREX_ESINGULAR, "view matrix %zu (projection %zu, sub-view %zu) is singular",
                        k, k / n_sub, k % n_sub);
        SubView &sv = tab[k];
        bool inside = true;
        for (int i = 0; i < 3; ++i) {
            const double s = -(Mi[i][0] * p[3] + Mi[i][1] * p[7] + Mi[i][2] * p[11]);
            sv.S[i] = s + half[i];
            inside = inside && sv.S[i] >= 0.0 && sv.S[i] <= 2.0 * half[i];
            for (int j = 0; j < 3; ++j) sv.Mi[3 * i + j] = Mi[i][j];
        }
        if (inside)
            return fail(c, CTREX_ESOURCE_INSIDE, "source of view matrix %zu lies inside the volume", k);
        sv.tau = 0.0;
        sv.pad[0] = sv.pad[1] = sv.pad[2] = 0.0;
    }
    // commit
    CTREX_HIP(c, hipDeviceSynchronize());
    if (c->d_tab && c->tab.size() < m) {
        CTREX_HIP(c, hipFree(c->d_tab));
        c->d_tab = nullptr;
    }
    if (!c->d_tab) CTREX_HIP(c, hipMalloc(&c->d_tab, sizeof(SubView) * m));
    CTREX_HIP(c, hipMemcpy(c->d_tab, tab.data(), sizeof(SubView) * m, hipMemcpyHostToDevice));
    if (c->d_P && c->P_cap < m) {
        CTREX_HIP(c, hipFree(c->d_P));
        c->d_P = nullptr;
    }
    if (!c->d_P) {
        CTREX_HIP(c, hipMalloc(&c->d_P, sizeof(double) * 12 * m));
        c->P_cap = m;
    }
    CTREX_HIP(c, hipMemcpy(c->d_P, P, sizeof(double) * 12 * m, hipMemcpyHostToDevice));
    if (c->d_U) {
        CTREX_HIP(c, hipFree(c->d_U));
        c->d_U = nullptr;
    }
    c->tab = std::move(tab);
    c->P_host.assign(P, P + 12 * m);
    c->have_cyl = false;   // its tables derive from the view matrices
    c->n_proj = n_proj;
    c->n_sub = n_sub;
    c->n_u = n_u;
    c->n_v = n_v;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->step = step;
    c->have_geom = true;
    c->d_vw = nullptr;   // weights of another volume layout are void
    c->generation++;
    c->w_cache.clear();
    return CTREX_OK;
}

int ctrex_set_motion(ctrex_ctx *c, const float *U_dev, int32_t gx, int32_t gy, int32_t gz,
                     const double *tau) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!U_dev) {
        CTREX_HIP(c, hipDeviceSynchronize());
        if (c->d_U) CTREX_HIP(c, hipFree(c->d_U));
        c->d_U = nullptr;
        for (auto &sv : c->tab) sv.tau = 0.0;
        CTREX_HIP(c, hipMemcpy(c->d_tab, c->tab.data(), sizeof(SubView) * c->tab.size(),
                               hipMemcpyHostToDevice));
        c->generation++;
        c->w_cache.clear();
        return CTREX_OK;
    }
    if (!tau) return fail(c, CTREX_EINVAL, "tau is NULL");
    if (gx < 2 || gy < 2 || gz < 2) return fail(c, CTREX_ESHAPE, "grid sides must be >= 2");
    if (static_cast<long long>(gx) * gy * gz >= (1ll << 28))
        return fail(c, CTREX_ESHAPE, "displacement grid too large");
    for (size_t k = 0; k < c->tab.size(); ++k)
        if (!std::isfinite(tau[k])) return fail(c, CTREX_EINVAL, "tau[%zu] is not finite", k);
    const size_t nodes = static_cast<size_t>(gx) * gy * gz;
    CTREX_HIP(c, hipDeviceSynchronize());
    if (c->d_U) {
        CTREX_HIP(c, hipFree(c->d_U));
        c->d_U = nullptr;
    }
    // bound of the displacement on every axis, for the backprojector's bricks
    std::vector<float> hostU(3 * nodes);
    CTREX_HIP(c, hipMemcpy(hostU.data(), U_dev, sizeof(float) * 3 * nodes, hipMemcpyDeviceToHost));
    double umax = 0.0, tmax = 0.0;
    for (float v : hostU) {
        if (!std::isfinite(v)) return fail(c, CTREX_EINVAL, "displacement grid is not finite");
        umax = std::max(umax, static_cast<double>(std::fabs(v)));
    }
    for (size_t k = 0; k < c->tab.size(); ++k) tmax = std::max(tmax, std::fabs(tau[k]));
    const double bound = umax * tmax;
    if (bound > 64.0) return fail(c, CTREX_EINVAL, "displacement bound %g exceeds 64 voxels", bound);
    CTREX_HIP(c, hipMalloc(&c->d_U, sizeof(float4) * nodes));
    CTREX_HIP(c, launch_repack_warp(U_dev, c->d_U, nodes, nullptr));
    c->warp_margin = static_cast<int>(std::ceil(bound * (1.0 + 1e-6) + 1e-6));
    c->warp_umax = umax;
    for (size_t k = 0; k < c->tab.size(); ++k) c->tab[k].tau = tau[k];
    CTREX_HIP(c, hipMemcpy(c->d_tab, c->tab.data(), sizeof(SubView) * c->tab.size(),
                           hipMemcpyHostToDevice));
    CTREX_HIP(c, hipDeviceSynchronize());
    c->gx = gx;
    c->gy = gy;
    c->gz = gz;
    c->generation++;
    c->w_cache.clear();
    return CTREX_OK;
}

int ctrex_set_voxel_weights(ctrex_ctx *c, const float *w_dev) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    c->d_vw = w_dev;
    return CTREX_OK;
}

int ctrex_forward_project(ctrex_ctx *c, const void *vol, int32_t vol_dtype, void *sino,
                          int32_t sino_dtype, const int32_t *views, int32_t n_views,
                          void *stream) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!valid_dtype(vol_dtype) || !valid_dtype(sino_dtype))
        return fail(c, CTREX_EINVAL, "unknown dtype (%d, %d)", vol_dtype, sino_dtype);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if (nv == 0) return CTREX_OK;  // nothing to project (pointers may be NULL)
    if (!vol || !sino) return fail(c, CTREX_EINVAL, "vol and sino must be device pointers");
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    const RayGrid g = make_grid(c, dv, nv);
    const ProjScratch SL = proj_scratch(c, nv);
    void *scr;
    if ((st = ctx_scratch(c, SL.shared + packed_bytes(c, vol_dtype), &scr))) return st;
    FpExtra ex{nullptr, nullptr, nullptr};
    if ((st = make_gather_copies(c, vol, vol_dtype, static_cast<char *>(scr) + SL.shared, ex, s)))
        return st;
    CTREX_HIP(c, launch_forward(g, make_warp(c), vol, vol_dtype, sino, sino_dtype, FP_PLAIN, ex, s));
    return CTREX_OK;
}

int ctrex_residual_norm(ctrex_ctx *c, const void *vol, int32_t vol_dtype, const void *sino,
                        int32_t sino_dtype, const int32_t *views, int32_t n_views, double *norm,
                        void *stream) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!norm) return fail(c, CTREX_EINVAL, "norm must be a host pointer");
    if (!valid_dtype(vol_dtype) || !valid_dtype(sino_dtype))
        return fail(c, CTREX_EINVAL, "unknown dtype (%d, %d)", vol_dtype, sino_dtype);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    *norm = 0.0;
    if (nv == 0) return CTREX_OK;
    if (!vol || !sino) return fail(c, CTREX_EINVAL, "vol and sino must be device pointers");
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    const RayGrid g = make_grid(c, dv, nv);
    const ProjScratch SL = proj_scratch(c, nv);
    void *scr;
    if ((st = ctx_scratch(c, SL.total, &scr))) return st;
    double *part = reinterpret_cast<double *>(static_cast<char *>(scr) + SL.partials);
    FpExtra ex{sino, nullptr, part};
    if ((st = make_gather_copies(c, vol, vol_dtype, static_cast<char *>(scr) + SL.shared, ex, s)))
        return st;
    // `out` is unused in this mode; the sinogram's storage type selects the kernel
    CTREX_HIP(c, launch_forward(g, make_warp(c), vol, vol_dtype, nullptr, sino_dtype, FP_RESIDUAL,
                                ex, s));
    CTREX_HIP(c, launch_sum_partials(part, g.total_blocks, part + g.total_blocks, s));
    double h = 0.0;
    CTREX_HIP(c, hipMemcpyAsync(&h, part + g.total_blocks, sizeof h, hipMemcpyDeviceToHost, s));
    CTREX_HIP(c, hipStreamSynchronize(s));
    *norm = std::sqrt(h);
    if (!std::isfinite(*norm)) return fail(c, CTREX_ENONFINITE, "the residual norm is not finite");
    return CTREX_OK;
}

}  // extern "C"

namespace {

// vol (+)= scale A^T sino: ctrex_back_project and ctrex_back_project_scaled.
int back_project_common(ctrex_ctx *c, const void *sino, int32_t sino_dtype, float scale,
                        float *vol, int32_t accumulate, const int32_t *views, int32_t n_views,
                        void *stream) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!vol) return fail(c, CTREX_EINVAL, "vol must be a device pointer");
    if (!valid_dtype(sino_dtype)) return fail(c, CTREX_EINVAL, "unknown dtype %d", sino_dtype);
    if (!std::isfinite(scale)) return fail(c, CTREX_EINVAL, "scale must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    if (nv > 0 && !sino) return fail(c, CTREX_EINVAL, "sino must be a device pointer");
    if (nv == 0) {
        if (!accumulate)
            CTREX_HIP(c, launch_fill_zero(vol, sizeof(float) * static_cast<size_t>(c->nx) * c->ny * c->nz, s));
        return CTREX_OK;
    }
    const RayGrid g = make_grid(c, dv, nv);
    const ProjScratch SL = proj_scratch(c, nv);
    // the backprojector's 64-bit integer volume, in the shared region
    const size_t work = back_scratch_bytes(g);
    void *scr = nullptr;
    if ((st = ctx_scratch(c, SL.shared + work, &scr))) return st;
    void *acc = static_cast<char *>(scr) + SL.shared;
    CTREX_HIP(c, launch_back(g, make_warp(c), c->d_P, sino, sino_dtype, vol, accumulate ? 1 : 0,
                             BP_PLAIN, c->d_scalar, acc, s, scale));
    return CTREX_OK;
}

}  // namespace

extern "C" {

int ctrex_back_project(ctrex_ctx *c, const void *sino, int32_t sino_dtype, float *vol,
                       int32_t accumulate, const int32_t *views, int32_t n_views, void *stream) {
    return back_project_common(c, sino, sino_dtype, 1.0f, vol, accumulate, views, n_views,
                               stream);
}

int ctrex_back_project_scaled(ctrex_ctx *c, const void *sino, int32_t sino_dtype, float scale,
                              float *vol, int32_t accumulate, const int32_t *views,
                              int32_t n_views, void *stream) {
    return back_project_common(c, sino, sino_dtype, scale, vol, accumulate, views, n_views,
                               stream);
}

int ctrex_back_project_noalloc(ctrex_ctx *c, const void *sino, int32_t sino_dtype, float *vol,
                               int32_t accumulate, const int32_t *views, int32_t n_views,
                               void *stream) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!vol) return fail(c, CTREX_EINVAL, "vol must be a device pointer");
    if (!valid_dtype(sino_dtype)) return fail(c, CTREX_EINVAL, "unknown dtype %d", sino_dtype);
    int32_t nv = c->n_proj;
    if (views) {
        if (n_views < 0) return fail(c, CTREX_ESHAPE, "n_views must be >= 0 (got %d)", n_views);
        if (static_cast<size_t>(n_views) * sizeof(int32_t) > kNoAllocViewBytes)
            return fail(c, CTREX_ESHAPE, "view list of %d entries exceeds the %zu this call holds",
                        n_views, kNoAllocViewBytes / sizeof(int32_t));
        for (int32_t k = 0; k < n_views; ++k)
            if (views[k] < 0 || views[k] >= c->n_proj)
                return fail(c, CTREX_ESHAPE, "views[%d] = %d outside [0, %d)", k, views[k],
                            c->n_proj);
        nv = n_views;
    }
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    if (nv > 0 && !sino) return fail(c, CTREX_EINVAL, "sino must be a device pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t vox = static_cast<size_t>(c->nx) * c->ny * c->nz;
    if (nv == 0) {
        if (!accumulate) CTREX_HIP(c, launch_fill_zero(vol, sizeof(float) * vox, s));
        return CTREX_OK;
    }
    if ((st = noalloc_setup(c)) != CTREX_OK) return st;
    unsigned char *base = static_cast<unsigned char *>(noalloc_ptr[c->device]);
    const int32_t *dv = nullptr;
    if (views) {
        // the list is read from the caller's (pageable) memory during the call
        CTREX_HIP(c, hipMemcpyAsync(base, views, sizeof(int32_t) * nv, hipMemcpyHostToDevice, s));
        CTREX_HIP(c, hipStreamSynchronize(s));
        dv = reinterpret_cast<const int32_t *>(base);
    }
    // as many projection chunks (each writing a partial volume) as the array holds
    const size_t slab_room = kNoAllocBytes - kNoAllocSlabs;
    const size_t fit = slab_room / (sizeof(float) * vox);
    const int cap = fit >= 2 ? static_cast<int>(std::min<size_t>(fit, 1u << 20)) : 1;
    const RayGrid g = make_grid(c, dv, nv);
    const size_t slabs = back_scratch_bytes(g, cap, true);
    if (slabs > slab_room)
        return fail(c, CTREX_ESHAPE, "partial volumes of %zu bytes exceed the %zu this call holds",
                    slabs, slab_room);
    float *rmax = reinterpret_cast<float *>(base + kNoAllocMaxAbs);
    float *part = slabs ? reinterpret_cast<float *>(base + kNoAllocSlabs) : nullptr;
    // the direct form of the backprojector: no volume-sized buffer
    CTREX_HIP(c, launch_back(g, make_warp(c), c->d_P, sino, sino_dtype, vol, accumulate ? 1 : 0,
                             BP_PLAIN, rmax, part, s, 1.0f, cap, true));
    return CTREX_OK;
}

// Detector sizes the voxel-driven backprojector's bilinear lookups support
// (2 x 2 footprint, 24-bit row products, 32-bit byte offsets per image).
static bool voxel_bp_detector_ok(const ctrex_ctx *c) {
    return c->n_u >= 2 && c->n_v >= 2 && c->n_u < (1 << 24) && c->n_v < (1 << 24) &&
           static_cast<long long>(c->n_u) * c->n_v < (1ll << 30);
}

int ctrex_back_project_voxel(ctrex_ctx *c, const void *sino, int32_t sino_dtype, float *vol,
                             int32_t accumulate, const int32_t *views, int32_t n_views,
                             void *stream) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!vol) return fail(c, CTREX_EINVAL, "vol must be a device pointer");
    if (!valid_dtype(sino_dtype)) return fail(c, CTREX_EINVAL, "unknown dtype %d", sino_dtype);
    if (c->d_U) return fail(c, CTREX_ESTATE, "the voxel-driven backprojector has no motion warp");
    if (!voxel_bp_detector_ok(c))
        return fail(c, CTREX_ESHAPE, "the voxel-driven backprojector needs 2 <= n_u, n_v < 2^24 "
                                     "and n_u n_v < 2^30");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if (nv > 0 && !sino) return fail(c, CTREX_EINVAL, "sino must be a device pointer");
    if (nv == 0) {
        if (!accumulate)
            CTREX_HIP(c, launch_fill_zero(vol, sizeof(float) * static_cast<size_t>(c->nx) * c->ny * c->nz, s));
        return CTREX_OK;
    }
    CTREX_HIP(c, launch_back_voxel(make_grid(c, dv, nv), c->d_P, sino, sino_dtype, vol,
                                   accumulate ? 1 : 0, 0, VoxelGrid{}, s));
    return CTREX_OK;
}

int ctrex_sirt_workspace_bytes(const ctrex_ctx *c, int32_t n_views, uint32_t flags,
                               size_t *bytes) {
    if (!c || !bytes) return CTREX_EINVAL;
    if (!c->have_geom) return CTREX_ESTATE;
    if (n_views <= 0) n_views = c->n_proj;
    (void)flags;   // the gather flags change only the context's scratch
    *bytes = sirt_layout(c, n_views).total;
    return CTREX_OK;
}

int ctrex_sirt_iterate(ctrex_ctx *c, float *vol, const void *sino, int32_t sino_dtype,
                       int32_t n_iter, float alpha, uint32_t flags, const int32_t *views,
                       int32_t n_views, void *workspace, size_t workspace_bytes,
                       double *resid_norms, void *stream) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!vol || !sino) return fail(c, CTREX_EINVAL, "vol and sino must be device pointers");
    if (!valid_dtype(sino_dtype)) return fail(c, CTREX_EINVAL, "unknown dtype %d", sino_dtype);
    if (n_iter < 0) return fail(c, CTREX_EINVAL, "n_iter must be >= 0");
    if (!std::isfinite(alpha)) return fail(c, CTREX_EINVAL, "alpha must be finite");
    const uint32_t known = CTREX_NONNEG | CTREX_BF16_GATHER | CTREX_F16_GATHER |
                           CTREX_RECOMPUTE_WEIGHTS | CTREX_VOXEL_BP;
    if (flags & ~known) return fail(c, CTREX_EINVAL, "unknown flags 0x%x", flags & ~known);
    const bool vbp = (flags & CTREX_VOXEL_BP) != 0;
    if (vbp && c->d_U)
        return fail(c, CTREX_ESTATE, "the voxel-driven backprojector has no motion warp");
    if (vbp && !voxel_bp_detector_ok(c))
        return fail(c, CTREX_ESHAPE, "the voxel-driven backprojector needs 2 <= n_u, n_v < 2^24 "
                                     "and n_u n_v < 2^30");
    if ((flags & CTREX_BF16_GATHER) && (flags & CTREX_F16_GATHER))
        return fail(c, CTREX_EINVAL, "BF16 and F16 gathers are exclusive");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    if (nv == 0) return fail(c, CTREX_ESHAPE, "empty view subset");
    const SirtLayout L = sirt_layout(c, nv);
    if (!workspace) return fail(c, CTREX_EWORKSPACE, "workspace is NULL");
    if (workspace_bytes < L.total)
        return fail(c, CTREX_EWORKSPACE, "workspace of %zu bytes < %zu needed", workspace_bytes,
                    L.total);
    if (n_iter == 0) return CTREX_OK;
    char *ws = static_cast<char *>(workspace);
    float *Rw = reinterpret_cast<float *>(ws + L.R);
    void *r = ws + L.r;
    float *Cw = reinterpret_cast<float *>(ws + L.C);
    double *partials = reinterpret_cast<double *>(ws + L.partials);
    double *resid = reinterpret_cast<double *>(ws + L.resid);
    const int gdt = (flags & CTREX_BF16_GATHER) ? BF16 : (flags & CTREX_F16_GATHER) ? F16 : F32;
    const RayGrid g = make_grid(c, dv, nv);
    // scratch: z, the 16-bit shadow, and the gather copies, whose region the
    // backprojector's integer volume reuses (the copies are rebuilt after the
    // update that follows it)
    const ProjScratch SL = proj_scratch(c, nv);
    const size_t work = vbp ? 0 : back_scratch_bytes(g);
    void *scr;
    if ((st = ctx_scratch(c, SL.shared + std::max(packed_bytes(c, gdt), work), &scr)) != CTREX_OK)
        return st;
    char *sc = static_cast<char *>(scr);
    float *z = reinterpret_cast<float *>(sc + SL.z);
    void *shadow = sc + SL.shadow;
    const size_t vox = static_cast<size_t>(c->nx) * c->ny * c->nz;
    const int rdt = sino_dtype;  // the correction image takes the data's storage type
    const WarpGrid w = make_warp(c);
    void *part = work ? sc + SL.shared : nullptr;

    // R and C for this geometry / motion / subset / workspace, kept between calls.
    auto same_key = [&](const ctrex_ctx::WeightKey &e) {
        return e.ws == workspace && e.gen == c->generation && e.all == (views == nullptr) &&
               e.kind == (vbp ? 1 : 0) &&
               (views == nullptr ||
                (static_cast<int32_t>(e.views.size()) == nv &&
                 std::memcmp(e.views.data(), views, sizeof(int32_t) * nv) == 0));
    };
    // the workspace's R and C are valid only under its own key; any other
    // entry naming this workspace is stale once we write into it
    auto hit = std::find_if(c->w_cache.begin(), c->w_cache.end(), same_key);
    const bool cached = hit != c->w_cache.end() && !(flags & CTREX_RECOMPUTE_WEIGHTS);
    if (!cached) {
        c->w_cache.erase(std::remove_if(c->w_cache.begin(), c->w_cache.end(),
                                        [&](const ctrex_ctx::WeightKey &e) {
                                            return e.ws == workspace;
                                        }),
                         c->w_cache.end());
        FpExtra none{nullptr, nullptr, nullptr};
        CTREX_HIP(c, launch_forward(g, w, nullptr, F32, Rw, F32, FP_RECIP_ONES, none, s));
        if (vbp)
            CTREX_HIP(c, launch_back_voxel(g, c->d_P, nullptr, F32, Cw, 0, 1, VoxelGrid{}, s));
        else
            CTREX_HIP(c, launch_back(g, w, c->d_P, nullptr, F32, Cw, 0, BP_ONES, c->d_scalar, part,
                                     s));
        CTREX_HIP(c, launch_recip(Cw, vox, s));
        ctrex_ctx::WeightKey k{workspace, c->generation, views == nullptr, vbp ? 1 : 0, {}};
        if (views) k.views.assign(views, views + nv);
        c->w_cache.insert(c->w_cache.begin(), std::move(k));
        if (c->w_cache.size() > kMaxWeightSets) c->w_cache.pop_back();
    } else if (hit != c->w_cache.begin()) {
        std::rotate(c->w_cache.begin(), hit, hit + 1);
    }
    const void *gather = vol;
    if (gdt != F32) {
        CTREX_HIP(c, launch_convert(vol, F32, shadow, gdt, vox, s));
        gather = shadow;
    }
    void *vt = sc + SL.shared;
    const bool packed = kPackedCorners && gdt == F32;
    const bool packed16 = kPacked16 && gdt != F32;
    float4 *p4 = static_cast<float4 *>(vt);
    uint2 *p2 = static_cast<uint2 *>(vt);
    auto refresh_copies = [&]() -> hipError_t {
        if (packed) return launch_pack_corners(vol, p4, p4 + vox, c->nx, c->ny, c->nz, s);
        if (packed16)
            return launch_pack_corners16(static_cast<const uint16_t *>(gather), p2, p2 + vox,
                                         c->nx, c->ny, c->nz, s);
        return launch_transpose_xy(gather, vt, gdt, c->nx, c->ny, c->nz, s);
    };
    CTREX_HIP(c, refresh_copies());
    std::vector<double> host_norms;
    if (resid_norms) host_norms.reserve(n_iter);
    FpExtra ex{sino, Rw, partials};
    if (packed) {
        ex.p4 = p4;
        ex.p4t = p4 + vox;
    } else if (packed16) {
        ex.p2 = p2;
        ex.p2t = p2 + vox;
    } else {
        ex.vol_t = vt;
    }
    for (int32_t k = 0; k < n_iter; ++k) {
        PhaseTimer t_fp{c, s, nullptr, 0}, t_bp{c, s, nullptr, 1}, t_up{c, s, nullptr, 2};
        CTREX_HIP(c, t_fp.begin());
        CTREX_HIP(c, launch_forward(g, w, gather, gdt, r, rdt, FP_CORRECT, ex, s));
        CTREX_HIP(c, t_fp.end());
        CTREX_HIP(c, launch_sum_partials(partials, g.total_blocks, resid + (k % kResidCap), s));
        CTREX_HIP(c, t_bp.begin());
        if (vbp)
            CTREX_HIP(c, launch_back_voxel(g, c->d_P, r, rdt, z, 0, 0, VoxelGrid{}, s));
        else
            CTREX_HIP(c, launch_back(g, w, c->d_P, r, rdt, z, 0, BP_PLAIN, c->d_scalar, part, s));
        CTREX_HIP(c, t_bp.end());
        CTREX_HIP(c, t_up.begin());
        CTREX_HIP(c, launch_update(vol, z, Cw, c->d_vw, alpha, (flags & CTREX_NONNEG) ? 1 : 0,
                                   gdt != F32 ? shadow : nullptr, gdt, vox, s));
        if (k + 1 < n_iter) CTREX_HIP(c, refresh_copies());
        CTREX_HIP(c, t_up.end());
        if (resid_norms && ((k + 1) % kResidCap == 0 || k + 1 == n_iter)) {
            const int cnt = (k % kResidCap) + 1;
            std::vector<double> tmp(cnt);
            CTREX_HIP(c, hipMemcpyAsync(tmp.data(), resid, sizeof(double) * cnt,
                                        hipMemcpyDeviceToHost, s));
            CTREX_HIP(c, hipStreamSynchronize(s));
            host_norms.insert(host_norms.end(), tmp.begin(), tmp.end());
        }
    }
    if (resid_norms) {
        bool finite = true;
        for (int32_t k = 0; k < n_iter; ++k) {
            resid_norms[k] = std::sqrt(host_norms[k]);
            finite = finite && std::isfinite(resid_norms[k]);
        }
        if (!finite) return fail(c, CTREX_ENONFINITE, "a residual norm is not finite");
    }
    return CTREX_OK;
}

int ctrex_sample_count(ctrex_ctx *c, const int32_t *views, int32_t n_views, int64_t *count,
                       void *stream) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!count) return fail(c, CTREX_EINVAL, "count is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    CTREX_HIP(c, launch_fill_zero(c->d_count, sizeof(unsigned long long), s));
    CTREX_HIP(c, launch_sample_count(make_grid(c, dv, nv), c->d_count, s));
    unsigned long long h = 0;
    CTREX_HIP(c, hipMemcpyAsync(&h, c->d_count, sizeof h, hipMemcpyDeviceToHost, s));
    CTREX_HIP(c, hipStreamSynchronize(s));
    *count = static_cast<int64_t>(h);
    return CTREX_OK;
}

int ctrex_tv(ctrex_ctx *c, const float *x, int32_t nx, int32_t ny, int32_t nz, float eps,
             float weight, double *value, float *grad, void *stream) {
    if (!c) return CTREX_EINVAL;
    if (!x) return fail(c, CTREX_EINVAL, "x must be a device pointer");
    if (nx < 1 || ny < 1 || nz < 1 || static_cast<long long>(nx) * ny * nz >= (1ll << 40))
        return fail(c, CTREX_ESHAPE, "bad volume shape");
    if (!(eps >= 0.0f) || !std::isfinite(eps) || !std::isfinite(weight))
        return fail(c, CTREX_EINVAL, "eps must be finite and >= 0, weight finite");
    if (grad == x) return fail(c, CTREX_EINVAL, "grad must not alias x");
    CTREX_HIP(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (grad) CTREX_HIP(c, launch_tv_grad(x, nx, ny, nz, eps, weight, grad, s));
    if (value) {
        const size_t n = static_cast<size_t>(nx) * ny * nz;
        const int blocks = tv_blocks(n);
        CTREX_HIP(c, launch_tv_value(x, nx, ny, nz, eps, c->d_red, s));
        CTREX_HIP(c, launch_sum_partials(c->d_red, blocks, c->d_red + 8192, s));
        CTREX_HIP(c, hipMemcpyAsync(value, c->d_red + 8192, sizeof(double), hipMemcpyDeviceToHost, s));
        CTREX_HIP(c, hipStreamSynchronize(s));
    }
    return CTREX_OK;
}

int ctrex_profile_enable(ctrex_ctx *c, int32_t enable) {
    if (!c) return CTREX_EINVAL;
    CTREX_HIP(c, hipSetDevice(c->device));
    CTREX_HIP(c, hipDeviceSynchronize());
    for (auto &m : c->ev_marks) {
        c->ev_pool.push_back(m.second.first);
        c->ev_pool.push_back(m.second.second);
    }
    c->ev_marks.clear();
    c->profiling = enable != 0;
    return CTREX_OK;
}

int ctrex_profile_read(ctrex_ctx *c, double *ms, int64_t *launches) {
    if (!c || !ms || !launches) return CTREX_EINVAL;
    CTREX_HIP(c, hipSetDevice(c->device));
    for (int i = 0; i < 3; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    for (auto &m : c->ev_marks) {
        CTREX_HIP(c, hipEventSynchronize(m.second.second));
        float t = 0.0f;
        CTREX_HIP(c, hipEventElapsedTime(&t, m.second.first, m.second.second));
        ms[m.first] += t;
        launches[m.first] += 1;
        c->ev_pool.push_back(m.second.first);
        c->ev_pool.push_back(m.second.second);
    }
    c->ev_marks.clear();
    return CTREX_OK;
}

int ctrex_convert(ctrex_ctx *c, const void *src, int32_t src_dtype, void *dst, int32_t dst_dtype,
                  int64_t n, void *stream) {
    if (!c) return CTREX_EINVAL;
    if (!src || !dst) return fail(c, CTREX_EINVAL, "src and dst must be device pointers");
    if (!valid_dtype(src_dtype) || !valid_dtype(dst_dtype))
        return fail(c, CTREX_EINVAL, "unknown dtype");
    if (n < 0) return fail(c, CTREX_ESHAPE, "n must be >= 0");
    CTREX_HIP(c, hipSetDevice(c->device));
    CTREX_HIP(c, launch_convert(src, src_dtype, dst, dst_dtype, static_cast<size_t>(n),
                                static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_scratch_bytes(const ctrex_ctx *c, int32_t n_views, size_t *bytes) {
    if (!c || !bytes) return CTREX_EINVAL;
    if (!c->have_geom) return CTREX_ESTATE;
    if (n_views <= 0) n_views = c->n_proj;
    size_t need = proj_scratch(c, n_views).total;
    if (c->have_cyl) need = std::max(need, cyl_scratch(c).total);
    *bytes = need;
    return CTREX_OK;
}

int ctrex_set_scratch(ctrex_ctx *c, void *dev, size_t bytes) {
    if (!c) return CTREX_EINVAL;
    if (!dev && bytes) return fail(c, CTREX_EINVAL, "NULL scratch with a non-zero size");
    if (reinterpret_cast<uintptr_t>(dev) % 256 != 0)
        return fail(c, CTREX_EINVAL, "scratch must be 256-byte aligned");
    c->user_scratch = bytes ? dev : nullptr;
    c->user_scratch_bytes = dev ? bytes : 0;
    return CTREX_OK;
}

int ctrex_data_residual(ctrex_ctx *c, const void *vol, int32_t vol_dtype, const void *b, void *r,
                        int32_t sino_dtype, float scale, const int32_t *views, int32_t n_views,
                        double *sq_sum, void *stream) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!valid_dtype(vol_dtype) || !valid_dtype(sino_dtype))
        return fail(c, CTREX_EINVAL, "unknown dtype (%d, %d)", vol_dtype, sino_dtype);
    if (!r && !sq_sum) return fail(c, CTREX_EINVAL, "neither r nor sq_sum requested");
    if (!std::isfinite(scale)) return fail(c, CTREX_EINVAL, "scale must be finite");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if (nv == 0) {
        if (sq_sum) CTREX_HIP(c, launch_fill_zero(sq_sum, sizeof(double), s));
        return CTREX_OK;
    }
    if (!vol || !b) return fail(c, CTREX_EINVAL, "vol and b must be device pointers");
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    const RayGrid g = make_grid(c, dv, nv);
    const ProjScratch SL = proj_scratch(c, nv);
    void *scr;
    if ((st = ctx_scratch(c, SL.total, &scr))) return st;
    double *part = reinterpret_cast<double *>(static_cast<char *>(scr) + SL.partials);
    // the correction epilogue without R stores rscale (b - A vol) = scale (A vol - b)
    FpExtra ex{b, nullptr, part};
    ex.rscale = -scale;
    if ((st = make_gather_copies(c, vol, vol_dtype, static_cast<char *>(scr) + SL.shared, ex, s)))
        return st;
    CTREX_HIP(c, launch_forward(g, make_warp(c), vol, vol_dtype, r, sino_dtype,
                                r ? FP_CORRECT : FP_RESIDUAL, ex, s));
    if (sq_sum) CTREX_HIP(c, launch_sum_partials(part, g.total_blocks, sq_sum, s));
    return CTREX_OK;
}

}  // extern "C"

// ------------------------------------------------ aligned cylindrical domain --

namespace {

int check_cyl_ready(ctrex_ctx *c) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (!c->have_cyl)
        return fail(c, CTREX_ESTATE, "no cylindrical domain set (call ctrex_set_cylinder)");
    if (c->d_U) return fail(c, CTREX_ESTATE, "the cylindrical domain has no motion warp");
    return CTREX_OK;
}

RayGrid make_grid_cyl(const ctrex_ctx *c, const int32_t *dev_views, int32_t n_views) {
    RayGrid g = make_grid(c, dev_views, n_views);
    g.tab = c->d_tab_cyl;
    g.nx = c->cyl_nr;
    g.ny = c->cyl_nphi;
    g.nz = c->cyl_nz;
    return g;
}

CylGrid cyl_of(const ctrex_ctx *c) {
    return make_cyl_grid(c->cyl_nr, c->cyl_nphi, c->cyl_nz, c->cyl_dr, c->cyl_dz);
}

VoxelGrid cyl_voxels(const ctrex_ctx *c) {
    VoxelGrid v;
    v.cyl = 1;
    v.dr = c->cyl_dr;
    v.dz = c->cyl_dz;
    return v;
}

// As for the Cartesian SIRT: the workspace keeps R, r, C and the partials;
// the correction volume and the packed copy live in the attached scratch.
struct CylLayout {
    size_t R, r, C, partials, resid, total;
};

CylLayout cyl_layout(const ctrex_ctx *c, int32_t n_views) {
    const size_t rays = static_cast<size_t>(n_views) * c->n_u * c->n_v;
    const size_t vox = static_cast<size_t>(c->cyl_nr) * c->cyl_nphi * c->cyl_nz;
    const size_t tiles = static_cast<size_t>((c->n_u + TILE_U - 1) / TILE_U) *
                         ((c->n_v + TILE_V - 1) / TILE_V) * n_views;
    CylLayout l;
    size_t off = 0;
    l.R = off;
    off = align_up(off + 4 * rays);
    l.r = off;
    off = align_up(off + 4 * rays);
    l.C = off;
    off = align_up(off + 4 * vox);
    l.partials = off;
    off = align_up(off + 8 * tiles);
    l.resid = off;
    off = align_up(off + 8 * kResidCap);
    l.total = off;
    return l;
}

}  // namespace

extern "C" {

int ctrex_set_cylinder(ctrex_ctx *c, int32_t n_r, int32_t n_phi, int32_t n_z, double dr,
                       double dz, const double *pose) {
    int st = check_ready(c);
    if (st != CTREX_OK) return st;
    if (n_r < 2 || n_phi < 3 || n_z < 2)
        return fail(c, CTREX_ESHAPE, "need n_r >= 2, n_phi >= 3, n_z >= 2");
    if (static_cast<long long>(n_r) * n_phi * n_z >= (1ll << 31))
        return fail(c, CTREX_ESHAPE, "cylindrical volume exceeds 2^31 - 1 voxels");
    if (!(dr > 0.0) || !(dz > 0.0) || !std::isfinite(dr) || !std::isfinite(dz))
        return fail(c, CTREX_EINVAL, "dr and dz must be finite and > 0");
    double R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, t[3] = {0, 0, 0};
    if (pose) {
        for (int i = 0; i < 12; ++i)
            if (!std::isfinite(pose[i])) return fail(c, CTREX_EINVAL, "pose is not finite");
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) R[i][j] = pose[4 * i + j];
            t[i] = pose[4 * i + 3];
        }
        // a rotation: R^T R = I and det R = +1
        double err = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double d = -(i == j ? 1.0 : 0.0);
                for (int k = 0; k < 3; ++k) d += R[k][i] * R[k][j];
                err = std::max(err, std::fabs(d));
            }
        double inv[3][3];
        if (err > 1e-9 || invert3(R, inv) < 0.0)
            return fail(c, CTREX_EINVAL, "pose is not a rotation plus translation");
    }
    const double rh = (n_r - 0.5) * dr, hz = 0.5 * (n_z - 1) * dz;
    if (std::sqrt(4.0 * rh * rh + 4.0 * hz * hz) / c->step >= double(1 << 24))
        return fail(c, CTREX_EINVAL, "step %g too small for the cylinder", c->step);
    const size_t m = static_cast<size_t>(c->n_proj) * c->n_sub;
    std::vector<SubView> tab(m);
    std::vector<double> Pc(12 * m);
    for (size_t k = 0; k < m; ++k) {
        const double *p = c->P_host.data() + 12 * k;
        double M[3][3], Mi[3][3], S[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = p[4 * i + j];
        (void)invert3(M, Mi);   // ctrex_set_geometry checked it is regular
        for (int i = 0; i < 3; ++i) S[i] = -(Mi[i][0] * p[3] + Mi[i][1] * p[7] + Mi[i][2] * p[11]);
        SubView &sv = tab[k];
        for (int i = 0; i < 3; ++i) {
            sv.S[i] = R[i][0] * S[0] + R[i][1] * S[1] + R[i][2] * S[2] + t[i];
            for (int j = 0; j < 3; ++j)
                sv.Mi[3 * i + j] = R[i][0] * Mi[0][j] + R[i][1] * Mi[1][j] + R[i][2] * Mi[2][j];
        }
        sv.tau = 0.0;
        sv.pad[0] = sv.pad[1] = sv.pad[2] = 0.0;
        if (sv.S[0] * sv.S[0] + sv.S[1] * sv.S[1] <= rh * rh && std::fabs(sv.S[2]) <= hz)
            return fail(c, CTREX_ESOURCE_INSIDE,
                        "source of view matrix %zu lies inside the cylinder", k);
        // P T^-1 with T^-1 = [R^T, -R^T t]: maps cylinder-frame points like P maps V-frame ones
        double *q = Pc.data() + 12 * k;
        for (int i = 0; i < 3; ++i) {
            double lin = p[4 * i + 3];
            for (int j = 0; j < 3; ++j) {
                double a = 0.0;
                for (int l = 0; l < 3; ++l) a += p[4 * i + l] * R[j][l];
                q[4 * i + j] = a;
                lin -= a * t[j];
            }
            q[4 * i + 3] = lin;
        }
    }
    CTREX_HIP(c, hipDeviceSynchronize());
    if (c->cyl_cap < m) {
        if (c->d_tab_cyl) CTREX_HIP(c, hipFree(c->d_tab_cyl));
        if (c->d_P_cyl) CTREX_HIP(c, hipFree(c->d_P_cyl));
        c->d_tab_cyl = nullptr;
        c->d_P_cyl = nullptr;
        c->cyl_cap = 0;
        CTREX_HIP(c, hipMalloc(&c->d_tab_cyl, sizeof(SubView) * m));
        CTREX_HIP(c, hipMalloc(&c->d_P_cyl, sizeof(double) * 12 * m));
        c->cyl_cap = m;
    }
    CTREX_HIP(c, hipMemcpy(c->d_tab_cyl, tab.data(), sizeof(SubView) * m, hipMemcpyHostToDevice));
    CTREX_HIP(c, hipMemcpy(c->d_P_cyl, Pc.data(), sizeof(double) * 12 * m, hipMemcpyHostToDevice));
    c->cyl_nr = n_r;
    c->cyl_nphi = n_phi;
    c->cyl_nz = n_z;
    c->cyl_dr = dr;
    c->cyl_dz = dz;
    c->have_cyl = true;
    c->generation++;
    c->w_cache.clear();
    return CTREX_OK;
}

int ctrex_forward_project_cyl(ctrex_ctx *c, const void *vol, int32_t vol_dtype, void *sino,
                              int32_t sino_dtype, const int32_t *views, int32_t n_views,
                              void *stream) {
    int st = check_cyl_ready(c);
    if (st != CTREX_OK) return st;
    if (!valid_dtype(vol_dtype) || !valid_dtype(sino_dtype))
        return fail(c, CTREX_EINVAL, "unknown dtype (%d, %d)", vol_dtype, sino_dtype);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if (nv == 0) return CTREX_OK;
    if (!vol || !sino) return fail(c, CTREX_EINVAL, "vol and sino must be device pointers");
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    FpExtra ex{nullptr, nullptr, nullptr};
    if (kPackedCorners && vol_dtype == F32) {
        const CylScratch CL = cyl_scratch(c);
        void *scr;
        if ((st = ctx_scratch(c, CL.total, &scr))) return st;
        float4 *pk = reinterpret_cast<float4 *>(static_cast<char *>(scr) + CL.packed);
        CTREX_HIP(c, launch_pack_polar(static_cast<const float *>(vol), pk, c->cyl_nr, c->cyl_nphi,
                                       c->cyl_nz, s));
        ex.p4 = pk;
    }
    CTREX_HIP(c, launch_forward_cyl(make_grid_cyl(c, dv, nv), cyl_of(c), vol, vol_dtype, sino,
                                    sino_dtype, FP_PLAIN, ex, s));
    return CTREX_OK;
}

int ctrex_back_project_cyl(ctrex_ctx *c, const void *sino, int32_t sino_dtype, float *vol,
                           int32_t accumulate, const int32_t *views, int32_t n_views,
                           void *stream) {
    int st = check_cyl_ready(c);
    if (st != CTREX_OK) return st;
    if (!vol) return fail(c, CTREX_EINVAL, "vol must be a device pointer");
    if (!valid_dtype(sino_dtype)) return fail(c, CTREX_EINVAL, "unknown dtype %d", sino_dtype);
    if (!voxel_bp_detector_ok(c))
        return fail(c, CTREX_ESHAPE, "the voxel-driven backprojector needs 2 <= n_u, n_v < 2^24 "
                                     "and n_u n_v < 2^30");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if (nv > 0 && !sino) return fail(c, CTREX_EINVAL, "sino must be a device pointer");
    if (nv == 0) {
        if (!accumulate)
            CTREX_HIP(c, launch_fill_zero(vol, sizeof(float) * static_cast<size_t>(c->cyl_nr) *
                                                   c->cyl_nphi * c->cyl_nz, s));
        return CTREX_OK;
    }
    CTREX_HIP(c, launch_back_voxel(make_grid_cyl(c, dv, nv), c->d_P_cyl, sino, sino_dtype, vol,
                                   accumulate ? 1 : 0, 0, cyl_voxels(c), s));
    return CTREX_OK;
}

int ctrex_sample_count_cyl(ctrex_ctx *c, const int32_t *views, int32_t n_views, int64_t *count,
                           void *stream) {
    int st = check_cyl_ready(c);
    if (st != CTREX_OK) return st;
    if (!count) return fail(c, CTREX_EINVAL, "count is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    CTREX_HIP(c, launch_fill_zero(c->d_count, sizeof(unsigned long long), s));
    CTREX_HIP(c, launch_sample_count_cyl(make_grid_cyl(c, dv, nv), cyl_of(c), c->d_count, s));
    unsigned long long h = 0;
    CTREX_HIP(c, hipMemcpyAsync(&h, c->d_count, sizeof h, hipMemcpyDeviceToHost, s));
    CTREX_HIP(c, hipStreamSynchronize(s));
    *count = static_cast<int64_t>(h);
    return CTREX_OK;
}

int ctrex_sirt_workspace_bytes_cyl(const ctrex_ctx *c, int32_t n_views, size_t *bytes) {
    if (!c || !bytes) return CTREX_EINVAL;
    if (!c->have_geom || !c->have_cyl) return CTREX_ESTATE;
    if (n_views <= 0) n_views = c->n_proj;
    *bytes = cyl_layout(c, n_views).total;
    return CTREX_OK;
}

int ctrex_sirt_iterate_cyl(ctrex_ctx *c, float *vol, const void *sino, int32_t sino_dtype,
                           int32_t n_iter, float alpha, uint32_t flags, const int32_t *views,
                           int32_t n_views, void *workspace, size_t workspace_bytes,
                           double *resid_norms, void *stream) {
    int st = check_cyl_ready(c);
    if (st != CTREX_OK) return st;
    if (!vol || !sino) return fail(c, CTREX_EINVAL, "vol and sino must be device pointers");
    if (!valid_dtype(sino_dtype)) return fail(c, CTREX_EINVAL, "unknown dtype %d", sino_dtype);
    if (n_iter < 0) return fail(c, CTREX_EINVAL, "n_iter must be >= 0");
    if (!std::isfinite(alpha)) return fail(c, CTREX_EINVAL, "alpha must be finite");
    const uint32_t known = CTREX_NONNEG | CTREX_RECOMPUTE_WEIGHTS;
    if (flags & ~known) return fail(c, CTREX_EINVAL, "unsupported flags 0x%x", flags & ~known);
    if (!voxel_bp_detector_ok(c))
        return fail(c, CTREX_ESHAPE, "the voxel-driven backprojector needs 2 <= n_u, n_v < 2^24 "
                                     "and n_u n_v < 2^30");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *dv;
    int32_t nv;
    if ((st = resolve_views(c, views, n_views, &dv, &nv, s)) != CTREX_OK) return st;
    if ((st = check_blocks(c, nv)) != CTREX_OK) return st;
    if (nv == 0) return fail(c, CTREX_ESHAPE, "empty view subset");
    const CylLayout L = cyl_layout(c, nv);
    if (!workspace) return fail(c, CTREX_EWORKSPACE, "workspace is NULL");
    if (workspace_bytes < L.total)
        return fail(c, CTREX_EWORKSPACE, "workspace of %zu bytes < %zu needed", workspace_bytes,
                    L.total);
    if (n_iter == 0) return CTREX_OK;
    char *ws = static_cast<char *>(workspace);
    float *Rw = reinterpret_cast<float *>(ws + L.R);
    void *r = ws + L.r;
    float *Cw = reinterpret_cast<float *>(ws + L.C);
    double *partials = reinterpret_cast<double *>(ws + L.partials);
    double *resid = reinterpret_cast<double *>(ws + L.resid);
    const size_t vox = static_cast<size_t>(c->cyl_nr) * c->cyl_nphi * c->cyl_nz;
    // scratch: the correction volume z, then the corner-packed copy
    const CylScratch CL = cyl_scratch(c);
    void *scr;
    if ((st = ctx_scratch(c, CL.total, &scr)) != CTREX_OK) return st;
    float *z = reinterpret_cast<float *>(static_cast<char *>(scr) + CL.z);
    const RayGrid g = make_grid_cyl(c, dv, nv);
    const CylGrid cg = cyl_of(c);
    const VoxelGrid vg = cyl_voxels(c);
    auto same_key = [&](const ctrex_ctx::WeightKey &e) {
        return e.ws == workspace && e.gen == c->generation && e.all == (views == nullptr) &&
               e.kind == 2 &&
               (views == nullptr ||
                (static_cast<int32_t>(e.views.size()) == nv &&
                 std::memcmp(e.views.data(), views, sizeof(int32_t) * nv) == 0));
    };
    auto hit = std::find_if(c->w_cache.begin(), c->w_cache.end(), same_key);
    const bool cached = hit != c->w_cache.end() && !(flags & CTREX_RECOMPUTE_WEIGHTS);
    if (!cached) {
        c->w_cache.erase(std::remove_if(c->w_cache.begin(), c->w_cache.end(),
                                        [&](const ctrex_ctx::WeightKey &e) {
                                            return e.ws == workspace;
                                        }),
                         c->w_cache.end());
        FpExtra none{nullptr, nullptr, nullptr};
        CTREX_HIP(c, launch_forward_cyl(g, cg, nullptr, F32, Rw, F32, FP_RECIP_ONES, none, s));
        CTREX_HIP(c, launch_back_voxel(g, c->d_P_cyl, nullptr, F32, Cw, 0, 1, vg, s));
        CTREX_HIP(c, launch_recip(Cw, vox, s));
        ctrex_ctx::WeightKey k{workspace, c->generation, views == nullptr, 2, {}};
        if (views) k.views.assign(views, views + nv);
        c->w_cache.insert(c->w_cache.begin(), std::move(k));
        if (c->w_cache.size() > kMaxWeightSets) c->w_cache.pop_back();
    } else if (hit != c->w_cache.begin()) {
        std::rotate(c->w_cache.begin(), hit, hit + 1);
    }
    std::vector<double> host_norms;
    if (resid_norms) host_norms.reserve(n_iter);
    FpExtra ex{sino, Rw, partials};
    float4 *p4 = kPackedCorners ? reinterpret_cast<float4 *>(static_cast<char *>(scr) + CL.packed)
                                : nullptr;
    ex.p4 = p4;
    for (int32_t k = 0; k < n_iter; ++k) {
        PhaseTimer t_fp{c, s, nullptr, 0}, t_bp{c, s, nullptr, 1}, t_up{c, s, nullptr, 2};
        CTREX_HIP(c, t_fp.begin());
        if (p4) CTREX_HIP(c, launch_pack_polar(vol, p4, c->cyl_nr, c->cyl_nphi, c->cyl_nz, s));
        CTREX_HIP(c, launch_forward_cyl(g, cg, vol, F32, r, sino_dtype, FP_CORRECT, ex, s));
        CTREX_HIP(c, t_fp.end());
        CTREX_HIP(c, launch_sum_partials(partials, g.total_blocks, resid + (k % kResidCap), s));
        CTREX_HIP(c, t_bp.begin());
        CTREX_HIP(c, launch_back_voxel(g, c->d_P_cyl, r, sino_dtype, z, 0, 0, vg, s));
        CTREX_HIP(c, t_bp.end());
        CTREX_HIP(c, t_up.begin());
        CTREX_HIP(c, launch_update(vol, z, Cw, nullptr, alpha, (flags & CTREX_NONNEG) ? 1 : 0,
                                   nullptr, F32, vox, s));
        CTREX_HIP(c, t_up.end());
        if (resid_norms && ((k + 1) % kResidCap == 0 || k + 1 == n_iter)) {
            const int cnt = (k % kResidCap) + 1;
            std::vector<double> tmp(cnt);
            CTREX_HIP(c, hipMemcpyAsync(tmp.data(), resid, sizeof(double) * cnt,
                                        hipMemcpyDeviceToHost, s));
            CTREX_HIP(c, hipStreamSynchronize(s));
            host_norms.insert(host_norms.end(), tmp.begin(), tmp.end());
        }
    }
    if (resid_norms) {
        bool finite = true;
        for (int32_t k = 0; k < n_iter; ++k) {
            resid_norms[k] = std::sqrt(host_norms[k]);
            finite = finite && std::isfinite(resid_norms[k]);
        }
        if (!finite) return fail(c, CTREX_ENONFINITE, "a residual norm is not finite");
    }
    return CTREX_OK;
}

}  // extern "C"
