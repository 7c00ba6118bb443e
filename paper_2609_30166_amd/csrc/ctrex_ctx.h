// Context of the C ABI, shared by the runtime translation units.
#pragma once

#include <cstdarg>
#include <cstdio>
#include <list>
#include <string>
#include <utility>
#include <vector>

#include "ctrex_internal.h"

namespace ctrex {

struct DeviceViewList {
    std::vector<int32_t> host;
    int32_t *dev = nullptr;
};

}  // namespace ctrex

struct ctrex_ctx {
    int device = 0;
    // forward projector gather: 0 direct (corner-packed copies), 1 LDS-staged
    // tubes (CTREX_FP_GATHER=lds at context creation)
    int fp_tube = 0;
    std::string err;
    // geometry
    bool have_geom = false;
    int n_proj = 0, n_sub = 0, n_u = 0, n_v = 0, nx = 0, ny = 0, nz = 0;
    double step = 0.0;
    std::vector<ctrex::SubView> tab;
    ctrex::SubView *d_tab = nullptr;
    double *d_P = nullptr;    // view matrices [n_proj * n_sub][12]
    size_t P_cap = 0;
    std::vector<double> P_host;  // the same, as set
    // aligned cylindrical domain (ctrex_set_cylinder)
    bool have_cyl = false;
    int cyl_nr = 0, cyl_nphi = 0, cyl_nz = 0;
    double cyl_dr = 0.0, cyl_dz = 0.0;
    ctrex::SubView *d_tab_cyl = nullptr;  // sources and R_p M^-1 in the cylinder frame
    double *d_P_cyl = nullptr;            // P T^-1: matrices acting on cylinder-frame points
    size_t cyl_cap = 0;
    uint64_t generation = 0;  // bumps on geometry or motion change
    // motion
    float4 *d_U = nullptr;
    const float *d_vw = nullptr;   // caller's voxel weights (weighted backprojection)
    int gx = 0, gy = 0, gz = 0;
    int warp_margin = 0;  // ceil(max |tau| * max |U component|)
    double warp_umax = 0.0;  // max |U component|
    // cached device view lists (most recent first)
    std::list<ctrex::DeviceViewList> lists;
    // small fixed-size device scratch, allocated by ctrex_create
    unsigned long long *d_count = nullptr;
    float *d_scalar = nullptr;  // max |r| of the backprojector's input
    double *d_red = nullptr;    // 8192 block partials + 1 result (TV value)
    // caller-owned device scratch for the per-call volume-sized intermediates
    // (ctrex_set_scratch); the library never allocates these itself
    void *user_scratch = nullptr;
    size_t user_scratch_bytes = 0;
    // SIRT weight cache: which workspaces hold valid R and C for which
    // (geometry generation, view list, backprojector); most recent first, a few entries so
    // ordered subsets (one workspace each) keep their weights
    struct WeightKey {
        const void *ws;
        uint64_t gen;
        bool all;
        int kind;       // 0: C = 1/(A^T 1); 1: C = 1/(B 1) voxel-driven; 2: cylindrical domain
        std::vector<int32_t> views;
    };
    std::vector<WeightKey> w_cache;
    // kernel timing (ctrex_profile_enable)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_marks;
};


namespace ctrex {

inline int fail(ctrex_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

inline int hip_fail(ctrex_ctx *c, hipError_t e, const char *what) {
    return fail(c, CTREX_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// The caller's scratch attached with ctrex_set_scratch, if it holds at least
// `bytes`; otherwise CTREX_EWORKSPACE naming the size needed.
int ctx_scratch(ctrex_ctx *c, size_t bytes, void **out);

}  // namespace ctrex

#define CTREX_HIP(ctx, expr)                                               \
    do {                                                                   \
        hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) return ::ctrex::hip_fail((ctx), e_, #expr);  \
    } while (0)
