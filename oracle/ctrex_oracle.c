/*
 * CPU FP64 oracle of the ray-driven projector pair — TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this file's library.  It shares no code, header or constant with
 * the HIP library; it is written to be read against the paper, not to be fast.
 *
 * What it computes (paper Sec. 2.2 geometry, Sec. 4.1 projection operator,
 * Sec. 3.1 / 4.2.1 displacement warp, Sec. 3.4 / 4.2.2 angular sub-samples):
 *
 *   For projection p, sub-view s and pixel (iu, iv):
 *     M = P[:, :3], source S = -M^-1 P[:, 3]          (the point P sends to 0)
 *     d = M^-1 (iu, iv, 1)^T, normalised               (ray to the pixel centre)
 *     the line S + t d is clipped to the voxel-centre hull [0, n_a - 1]^3 of
 *     the index coordinates c = X + (n - 1)/2 (slab method) -> [t_in, t_out],
 *     L = t_out - t_in, n = ceil(L / step), h = L / n   (midpoint rule)
 *     samples c_i = S + (t_in + (i + 1/2) h) d, i = 0..n-1
 *     optional warp: c_i' = c_i + tau_{p,s} U(c_i); a warped sample outside
 *     the hull contributes nothing
 *     y[p, iv, iu] = (1 / n_sub) sum_s sum_i h * trilinear(x, c_i')
 *
 *   The backprojector is the exact transpose: every sample scatters
 *   (h / n_sub) * r[p, iv, iu] times its eight trilinear weights.
 *
 * Readings where the paper is silent: uniform Euclidean step adjusted per ray
 * (instead of dominant-axis slices), integration over the voxel-centre hull,
 * path-length weight h per sample, one ray per pixel centre, the mean over
 * sub-views, and a pull-back warp evaluated at the undeformed sample.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ESINGULAR (-3)
#define OR_ESOURCE_INSIDE (-4)

typedef struct {
    double S[3];    /* source in index coordinates (x, y, z) */
    double Mi[9];   /* inverse of P[:, :3], row-major */
    double tau;     /* time fraction of the sub-view (warp scale) */
} view_t;

typedef struct {
    int nx, ny, nz;
    const double *U;  /* [gz][gy][gx][3] displacement grid or NULL */
    int gx, gy, gz;
} warp_t;

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Source position and inverse matrix of one 3x4 view matrix (Sec. 2.2.1). */
static int view_setup(const double *P, const int n[3], double tau, view_t *v)
{
    const double a = P[0], b = P[1], c = P[2];
    const double d = P[4], e = P[5], f = P[6];
    const double g = P[8], h = P[9], i = P[10];
    double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
    double fro = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            fro += P[4 * r + k] * P[4 * r + k];
    fro = sqrt(fro);
    if (!(fro > 0.0) || !(fabs(det) >= 1e-12 * fro * fro * fro))
        return OR_ESINGULAR;
    /* inverse = adjugate / det */
    v->Mi[0] = (e * i - f * h) / det;
    v->Mi[1] = (c * h - b * i) / det;
    v->Mi[2] = (b * f - c * e) / det;
    v->Mi[3] = (f * g - d * i) / det;
    v->Mi[4] = (a * i - c * g) / det;
    v->Mi[5] = (c * d - a * f) / det;
    v->Mi[6] = (d * h - e * g) / det;
    v->Mi[7] = (b * g - a * h) / det;
    v->Mi[8] = (a * e - b * d) / det;
    int inside = 1;
    for (int r = 0; r < 3; ++r) {
        double s = -(v->Mi[3 * r] * P[3] + v->Mi[3 * r + 1] * P[7] + v->Mi[3 * r + 2] * P[11]);
        v->S[r] = s + 0.5 * (n[r] - 1); /* centred V frame -> index coordinates */
        if (v->S[r] < 0.0 || v->S[r] > (double)(n[r] - 1))
            inside = 0;
    }
    if (inside)
        return OR_ESOURCE_INSIDE;
    v->tau = tau;
    return OR_OK;
}

/* Unit direction of the ray through pixel (u, v). */
static void ray_direction(const view_t *v, double u, double w, double dir[3])
{
    double len = 0.0;
    for (int r = 0; r < 3; ++r) {
        dir[r] = v->Mi[3 * r] * u + v->Mi[3 * r + 1] * w + v->Mi[3 * r + 2];
        len += dir[r] * dir[r];
    }
    len = sqrt(len);
    for (int r = 0; r < 3; ++r)
        dir[r] /= len;
}

/* Slab clipping of S + t dir against [0, n_a - 1] on every axis. */
static int clip_hull(const double S[3], const double dir[3], const int n[3],
                     double *t_in, double *t_out)
{
    double lo_t = -INFINITY, hi_t = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double lo = 0.0, hi = (double)(n[a] - 1);
        if (dir[a] == 0.0) {
            if (S[a] < lo || S[a] > hi)
                return 0;
            continue;
        }
        double t1 = (lo - S[a]) / dir[a];
        double t2 = (hi - S[a]) / dir[a];
        double tmin = t1 < t2 ? t1 : t2;
        double tmax = t1 < t2 ? t2 : t1;
        if (tmin > lo_t) lo_t = tmin;
        if (tmax < hi_t) hi_t = tmax;
    }
    *t_in = lo_t;
    *t_out = hi_t;
    return hi_t > lo_t;
}

/* Lower corner and fraction of a coordinate on an axis of n >= 2 nodes. */
static void corner(double c, int n, int *i0, double *f)
{
    if (c < 0.0) c = 0.0;
    if (c > (double)(n - 1)) c = (double)(n - 1);
    int k = (int)floor(c);
    if (k > n - 2) k = n - 2;
    *i0 = k;
    *f = c - (double)k;
}

/* Trilinear interpolation of a [nz][ny][nx] array with `comp` values per node. */
static double trilinear(const double *vol, int nx, int ny, int nz, int comp, int which,
                        const double c[3])
{
    int ix, iy, iz;
    double fx, fy, fz;
    corner(c[0], nx, &ix, &fx);
    corner(c[1], ny, &iy, &fy);
    corner(c[2], nz, &iz, &fz);
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? fx : 1.0 - fx) * (dy ? fy : 1.0 - fy) * (dz ? fz : 1.0 - fz);
                size_t idx = ((size_t)(iz + dz) * ny + (iy + dy)) * nx + (ix + dx);
                acc += w * vol[idx * comp + which];
            }
    return acc;
}

/* Transpose of trilinear(): add val times the eight weights. */
static void trilinear_scatter(double *vol, int nx, int ny, int nz, const double c[3], double val)
{
    int ix, iy, iz;
    double fx, fy, fz;
    corner(c[0], nx, &ix, &fx);
    corner(c[1], ny, &iy, &fy);
    corner(c[2], nz, &iz, &fz);
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? fx : 1.0 - fx) * (dy ? fy : 1.0 - fy) * (dz ? fz : 1.0 - fz);
                size_t idx = ((size_t)(iz + dz) * ny + (iy + dy)) * nx + (ix + dx);
#pragma omp atomic
                vol[idx] += w * val;
            }
}

/* Pull-back warp of a sample (Sec. 3.1): c' = c + tau U(c).  The grid nodes span
 * the hull (node k of an axis sits at c = k (n-1)/(g-1)); lookups are clamped
 * to the grid.  Returns 0 when the warped sample leaves the hull. */
static int warp_sample(const warp_t *w, double tau, double c[3])
{
    if (!w->U)
        return 1;
    const int n[3] = {w->nx, w->ny, w->nz};
    const int g[3] = {w->gx, w->gy, w->gz};
    double gc[3];
    for (int a = 0; a < 3; ++a)
        gc[a] = c[a] * (double)(g[a] - 1) / (double)(n[a] - 1);
    double disp[3];
    for (int comp = 0; comp < 3; ++comp)
        disp[comp] = trilinear(w->U, w->gx, w->gy, w->gz, 3, comp, gc);
    for (int a = 0; a < 3; ++a) {
        c[a] += tau * disp[a];
        if (c[a] < 0.0 || c[a] > (double)(n[a] - 1))
            return 0;
    }
    return 1;
}

static int build_views(const double *P, int n_proj, int n_sub, const int n[3],
                       const double *tau, view_t **out)
{
    view_t *tab = (view_t *)malloc(sizeof(view_t) * (size_t)n_proj * n_sub);
    if (!tab)
        return OR_EINVAL;
    for (int k = 0; k < n_proj * n_sub; ++k) {
        int st = view_setup(P + 12 * (size_t)k, n, tau ? tau[k] : 0.0, &tab[k]);
        if (st != OR_OK) {
            free(tab);
            return st;
        }
    }
    *out = tab;
    return OR_OK;
}

static int check_dims(int n_proj, int n_sub, int nu, int nv, int nx, int ny, int nz, double step,
                      const int *views, int n_views)
{
    if (n_proj < 1 || n_sub < 1 || nu < 1 || nv < 1 || nx < 2 || ny < 2 || nz < 2)
        return OR_EINVAL;
    if (!(step > 0.0) || n_views < 0)
        return OR_EINVAL;
    if (views)
        for (int k = 0; k < n_views; ++k)
            if (views[k] < 0 || views[k] >= n_proj)
                return OR_EINVAL;
    return OR_OK;
}

/*
 * Forward projection.  P: [n_proj][n_sub][3][4]; vol: [nz][ny][nx];
 * views: n_views projection indices (NULL = 0..n_proj-1, n_views = n_proj);
 * sino: [n_views][nv][nu] output; U/tau optional warp; *n_samples = total
 * number of ray samples (warped-out samples included).
 */
int oracle_forward(const double *P, int n_proj, int n_sub, int nu, int nv,
                   int nx, int ny, int nz, double step, const double *vol,
                   const int *views, int n_views, const double *U, int gx, int gy, int gz,
                   const double *tau, double *sino, int64_t *n_samples)
{
    if (!views)
        n_views = n_proj;
    int st = check_dims(n_proj, n_sub, nu, nv, nx, ny, nz, step, views, n_views);
    if (st != OR_OK)
        return st;
    if (U && (gx < 2 || gy < 2 || gz < 2 || !tau))
        return OR_EINVAL;
    const int n[3] = {nx, ny, nz};
    view_t *tab;
    st = build_views(P, n_proj, n_sub, n, tau, &tab);
    if (st != OR_OK)
        return st;
    warp_t w = {nx, ny, nz, U, gx, gy, gz};
    int64_t total = 0;
#pragma omp parallel for collapse(2) schedule(dynamic, 4) reduction(+ : total)
    for (int k = 0; k < n_views; ++k) {
        for (int iv = 0; iv < nv; ++iv) {
            int p = views ? views[k] : k;
            for (int iu = 0; iu < nu; ++iu) {
                double acc = 0.0;
                for (int s = 0; s < n_sub; ++s) {
                    const view_t *v = &tab[(size_t)p * n_sub + s];
                    double dir[3], t_in, t_out;
                    ray_direction(v, (double)iu, (double)iv, dir);
                    if (!clip_hull(v->S, dir, n, &t_in, &t_out))
                        continue;
                    double L = t_out - t_in;
                    int64_t ns = (int64_t)ceil(L / step);
                    double h = L / (double)ns;
                    total += ns;
                    for (int64_t i = 0; i < ns; ++i) {
                        double t = t_in + ((double)i + 0.5) * h;
                        double c[3] = {v->S[0] + t * dir[0], v->S[1] + t * dir[1], v->S[2] + t * dir[2]};
                        if (!warp_sample(&w, v->tau, c))
                            continue;
                        acc += h * trilinear(vol, nx, ny, nz, 1, 0, c);
                    }
                }
                sino[((size_t)k * nv + iv) * nu + iu] = acc / (double)n_sub;
            }
        }
    }
    free(tab);
    if (n_samples)
        *n_samples = total;
    return OR_OK;
}

/* Backprojection, the exact transpose of oracle_forward: vol += A^T sino. */
int oracle_back(const double *P, int n_proj, int n_sub, int nu, int nv,
                int nx, int ny, int nz, double step, const double *sino,
                const int *views, int n_views, const double *U, int gx, int gy, int gz,
                const double *tau, double *vol)
{
    if (!views)
        n_views = n_proj;
    int st = check_dims(n_proj, n_sub, nu, nv, nx, ny, nz, step, views, n_views);
    if (st != OR_OK)
        return st;
    if (U && (gx < 2 || gy < 2 || gz < 2 || !tau))
        return OR_EINVAL;
    const int n[3] = {nx, ny, nz};
    view_t *tab;
    st = build_views(P, n_proj, n_sub, n, tau, &tab);
    if (st != OR_OK)
        return st;
    warp_t w = {nx, ny, nz, U, gx, gy, gz};
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int k = 0; k < n_views; ++k) {
        for (int iv = 0; iv < nv; ++iv) {
            int p = views ? views[k] : k;
            for (int iu = 0; iu < nu; ++iu) {
                double r = sino[((size_t)k * nv + iv) * nu + iu];
                for (int s = 0; s < n_sub; ++s) {
                    const view_t *v = &tab[(size_t)p * n_sub + s];
                    double dir[3], t_in, t_out;
                    ray_direction(v, (double)iu, (double)iv, dir);
                    if (!clip_hull(v->S, dir, n, &t_in, &t_out))
                        continue;
                    double L = t_out - t_in;
                    int64_t ns = (int64_t)ceil(L / step);
                    double h = L / (double)ns;
                    for (int64_t i = 0; i < ns; ++i) {
                        double t = t_in + ((double)i + 0.5) * h;
                        double c[3] = {v->S[0] + t * dir[0], v->S[1] + t * dir[1], v->S[2] + t * dir[2]};
                        if (!warp_sample(&w, v->tau, c))
                            continue;
                        trilinear_scatter(vol, nx, ny, nz, c, h * r / (double)n_sub);
                    }
                }
            }
        }
    }
    free(tab);
    return OR_OK;
}

/*
 * The same ray sampler with the trilinear lookup replaced by the indicator of
 * one ellipsoid ||Q (c - centre)|| <= 1 (index coordinates).  Used to pin the
 * sample positions and path-length weights against exact chord lengths.
 */
int oracle_forward_indicator(const double *P, int n_proj, int n_sub, int nu, int nv,
                             int nx, int ny, int nz, double step, const double *Q,
                             const double *centre, double *sino)
{
    int st = check_dims(n_proj, n_sub, nu, nv, nx, ny, nz, step, NULL, n_proj);
    if (st != OR_OK)
        return st;
    const int n[3] = {nx, ny, nz};
    view_t *tab;
    st = build_views(P, n_proj, n_sub, n, NULL, &tab);
    if (st != OR_OK)
        return st;
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int p = 0; p < n_proj; ++p) {
        for (int iv = 0; iv < nv; ++iv) {
            for (int iu = 0; iu < nu; ++iu) {
                double acc = 0.0;
                for (int s = 0; s < n_sub; ++s) {
                    const view_t *v = &tab[(size_t)p * n_sub + s];
                    double dir[3], t_in, t_out;
                    ray_direction(v, (double)iu, (double)iv, dir);
                    if (!clip_hull(v->S, dir, n, &t_in, &t_out))
                        continue;
                    double L = t_out - t_in;
                    int64_t ns = (int64_t)ceil(L / step);
                    double h = L / (double)ns;
                    for (int64_t i = 0; i < ns; ++i) {
                        double t = t_in + ((double)i + 0.5) * h;
                        double q2 = 0.0;
                        for (int r = 0; r < 3; ++r) {
                            double qr = 0.0;
                            for (int a = 0; a < 3; ++a)
                                qr += Q[3 * r + a] * (v->S[a] + t * dir[a] - centre[a]);
                            q2 += qr * qr;
                        }
                        if (q2 <= 1.0)
                            acc += h;
                    }
                }
                sino[((size_t)p * nv + iv) * nu + iu] = acc / (double)n_sub;
            }
        }
    }
    free(tab);
    return OR_OK;
}

/*
 * The paper's voxel-driven backprojector (Sec. 4.1, backprojection operator),
 * an unmatched alternative to the exact transpose: for voxel j with centre
 * X_j in the V frame and every listed projection p and sub-view s, the
 * detector point (u, v) with P (X_j, 1)^T proportional to (u, v, 1)^T samples
 * the correction image bilinearly (pixel centres at integer u, v; pixels
 * outside the detector count as zero):
 *     z_j = sum_p (1 / n_sub) sum_s r_p(u, v).
 * A point with a zero third component (in the source's detector-parallel
 * plane) contributes nothing.  No path-length weight: the SIRT normalisation
 * C = 1 / (B 1) absorbs the coverage (the paper's geometry-dependent
 * normalisation).
 */
static double bilinear_image(const double *img, int nu, int nv, double u, double v)
{
    /* every corner lies outside unless -1 < u < nu and -1 < v < nv (this also
     * keeps the integer conversions below in range) */
    if (!(u > -1.0 && u < nu && v > -1.0 && v < nv))
        return 0.0;
    double fu0 = floor(u), fv0 = floor(v);
    int u0 = (int)fu0, v0 = (int)fv0;
    double fu = u - fu0, fv = v - fv0;
    double acc = 0.0;
    for (int dv = 0; dv < 2; ++dv) {
        for (int du = 0; du < 2; ++du) {
            int iu = u0 + du, iv = v0 + dv;
            if (iu < 0 || iu >= nu || iv < 0 || iv >= nv)
                continue;
            double wgt = (du ? fu : 1.0 - fu) * (dv ? fv : 1.0 - fv);
            acc += wgt * img[(size_t)iv * nu + iu];
        }
    }
    return acc;
}

/* z_j for the voxel with centre (X, Y, Z) in the V frame. */
static double voxel_sum(const double *P, int n_sub, int nu, int nv, const double *sino,
                        const int *views, int n_views, double X, double Y, double Z)
{
    double acc = 0.0;
    for (int k = 0; k < n_views; ++k) {
        int p = views ? views[k] : k;
        const double *img = sino + (size_t)k * nu * nv;
        for (int s = 0; s < n_sub; ++s) {
            const double *M = P + 12 * ((size_t)p * n_sub + s);
            double a = M[0] * X + M[1] * Y + M[2] * Z + M[3];
            double b = M[4] * X + M[5] * Y + M[6] * Z + M[7];
            double w = M[8] * X + M[9] * Y + M[10] * Z + M[11];
            if (w == 0.0)
                continue;
            acc += bilinear_image(img, nu, nv, a / w, b / w) / (double)n_sub;
        }
    }
    return acc;
}

static int check_voxel_args(int n_proj, int n_sub, int nu, int nv, int nx, int ny, int nz,
                            const int *views, int n_views)
{
    if (n_proj < 1 || n_sub < 1 || nu < 1 || nv < 1 || nx < 1 || ny < 1 || nz < 1 || n_views < 0)
        return OR_EINVAL;
    for (int k = 0; k < n_views; ++k)
        if (views && (views[k] < 0 || views[k] >= n_proj))
            return OR_EINVAL;
    return OR_OK;
}

int oracle_back_voxel(const double *P, int n_proj, int n_sub, int nu, int nv, int nx, int ny,
                      int nz, const double *sino, const int *views, int n_views, double *vol)
{
    if (!views)
        n_views = n_proj;
    int st = check_voxel_args(n_proj, n_sub, nu, nv, nx, ny, nz, views, n_views);
    if (st != OR_OK)
        return st;
    const double ox = 0.5 * (nx - 1), oy = 0.5 * (ny - 1), oz = 0.5 * (nz - 1);
#pragma omp parallel for collapse(2) schedule(static)
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix)
                vol[((size_t)iz * ny + iy) * nx + ix] +=
                    voxel_sum(P, n_sub, nu, nv, sino, views, n_views, ix - ox, iy - oy, iz - oz);
    return OR_OK;
}

/* The same sums for a list of voxels (ix, iy, iz) only: out[i] = z_{j_i}. */
int oracle_back_voxel_points(const double *P, int n_proj, int n_sub, int nu, int nv, int nx,
                             int ny, int nz, const double *sino, const int *views, int n_views,
                             const int *ijk, int n_pts, double *out)
{
    if (!views)
        n_views = n_proj;
    int st = check_voxel_args(n_proj, n_sub, nu, nv, nx, ny, nz, views, n_views);
    if (st != OR_OK)
        return st;
    for (int i = 0; i < n_pts; ++i)
        if (ijk[3 * i] < 0 || ijk[3 * i] >= nx || ijk[3 * i + 1] < 0 || ijk[3 * i + 1] >= ny ||
            ijk[3 * i + 2] < 0 || ijk[3 * i + 2] >= nz)
            return OR_EINVAL;
    const double ox = 0.5 * (nx - 1), oy = 0.5 * (ny - 1), oz = 0.5 * (nz - 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n_pts; ++i)
        out[i] = voxel_sum(P, n_sub, nu, nv, sino, views, n_views, ijk[3 * i] - ox,
                           ijk[3 * i + 1] - oy, ijk[3 * i + 2] - oz);
    return OR_OK;
}

/*
 * Aligned cylindrical volume domain (Sec. 3.5 aligned cylindrical coordinates;
 * the projector's geometry-level modification and the backprojector's
 * counterpart, Sec. 4.2.1 / 4.3.1).
 *
 * The volume lives on a polar grid about the z axis of a cylinder frame.  A
 * point X of the V frame (the frame the view matrices act on, centred voxel
 * units) has cylinder-frame coordinates Xc = Rp X + tp for a rigid pose
 * [Rp | tp] (identity when none is given), and there
 *     r = sqrt(xc^2 + yc^2),  phi = atan2(yc, xc),  z = zc.
 * Grid nodes: ring i at r_i = (i + 1/2) dr (i < n_r), angle j at
 * phi_j = 2 pi j / n_phi (periodic), slice k at z_k = (k - (n_z - 1)/2) dz;
 * the volume is stored [n_z][n_phi][n_r], r fastest.  Continuous indices
 *     a = r / dr - 1/2 (clamped to [0, n_r - 1]: the core r < dr/2 takes the
 *         innermost ring's values), b = phi n_phi / (2 pi) mod n_phi,
 *     c = z / dz + (n_z - 1)/2,
 * and the value is trilinear in (a, b, c) with b periodic.  Rays are those of
 * the Cartesian projector (source S = -M^-1 P[:, 3], direction M^-1 (u, v, 1)
 * normalised, in the V frame), clipped to the hull r <= (n_r - 1/2) dr,
 * |z| <= (n_z - 1) dz / 2 in place of the box, and sampled at the midpoints of
 * n = ceil(L / step) equal parts, each weighted h = L / n; sub-views averaged.
 * The backprojector is the voxel-driven one of the Cartesian case with the
 * voxel centres (r_i cos phi_j, r_i sin phi_j, z_k) mapped back to the V frame,
 * X = Rp^T (Xc - tp).
 */
typedef struct {
    int nr, nphi, nz;
    double dr, dz;
    double R[9], t[3];   /* V frame -> cylinder frame */
} cyl_t;

static int cyl_init(cyl_t *c, int nr, int nphi, int nz, double dr, double dz, const double *pose)
{
    if (nr < 2 || nphi < 3 || nz < 2 || !(dr > 0.0) || !(dz > 0.0))
        return OR_EINVAL;
    c->nr = nr;
    c->nphi = nphi;
    c->nz = nz;
    c->dr = dr;
    c->dz = dz;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k)
            c->R[3 * r + k] = pose ? pose[4 * r + k] : (r == k ? 1.0 : 0.0);
        c->t[r] = pose ? pose[4 * r + 3] : 0.0;
    }
    return OR_OK;
}

static void cyl_frame(const cyl_t *c, const double X[3], double Xc[3])
{
    for (int r = 0; r < 3; ++r)
        Xc[r] = c->R[3 * r] * X[0] + c->R[3 * r + 1] * X[1] + c->R[3 * r + 2] * X[2] + c->t[r];
}

static double cyl_rh(const cyl_t *c) { return (c->nr - 0.5) * c->dr; }
static double cyl_hz(const cyl_t *c) { return 0.5 * (c->nz - 1) * c->dz; }

/* Trilinear value of the polar grid at cylinder-frame point Xc. */
static double cyl_value(const cyl_t *c, const double *vol, const double Xc[3])
{
    const double two_pi = 6.283185307179586476925287;
    double r = sqrt(Xc[0] * Xc[0] + Xc[1] * Xc[1]);
    double a = r / c->dr - 0.5;
    if (a < 0.0) a = 0.0;
    if (a > c->nr - 1) a = c->nr - 1;
    double b = atan2(Xc[1], Xc[0]) / two_pi * c->nphi;
    if (b < 0.0) b += c->nphi;
    double z = Xc[2] / c->dz + 0.5 * (c->nz - 1);
    if (z < 0.0) z = 0.0;
    if (z > c->nz - 1) z = c->nz - 1;
    int a0 = (int)floor(a), k0 = (int)floor(z), j0 = (int)floor(b);
    if (a0 > c->nr - 2) a0 = c->nr - 2;
    if (k0 > c->nz - 2) k0 = c->nz - 2;
    double fa = a - a0, fz = z - k0, fb = b - floor(b);
    if (j0 >= c->nphi) j0 -= c->nphi;
    int j1 = j0 + 1 == c->nphi ? 0 : j0 + 1;
    double acc = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int da = 0; da < 2; ++da) {
                double w = (da ? fa : 1.0 - fa) * (dj ? fb : 1.0 - fb) * (dk ? fz : 1.0 - fz);
                int j = dj ? j1 : j0;
                acc += w * vol[((size_t)(k0 + dk) * c->nphi + j) * c->nr + a0 + da];
            }
    return acc;
}

/* Clip the line Sc + t dc (cylinder frame) to the hull; 0 if it misses. */
static int cyl_clip(const cyl_t *c, const double Sc[3], const double dc[3], double *t0, double *t1)
{
    double lo = -INFINITY, hi = INFINITY;
    double Rh = cyl_rh(c), Hz = cyl_hz(c);
    double A = dc[0] * dc[0] + dc[1] * dc[1];
    double B = Sc[0] * dc[0] + Sc[1] * dc[1];
    double C = Sc[0] * Sc[0] + Sc[1] * Sc[1] - Rh * Rh;
    if (A == 0.0) {
        if (C > 0.0)
            return 0;
    } else {
        double disc = B * B - A * C;
        if (disc < 0.0)
            return 0;
        double sq = sqrt(disc);
        lo = (-B - sq) / A;
        hi = (-B + sq) / A;
    }
    if (dc[2] == 0.0) {
        if (fabs(Sc[2]) > Hz)
            return 0;
    } else {
        double za = (-Hz - Sc[2]) / dc[2], zb = (Hz - Sc[2]) / dc[2];
        double zmin = za < zb ? za : zb, zmax = za < zb ? zb : za;
        if (zmin > lo) lo = zmin;
        if (zmax < hi) hi = zmax;
    }
    *t0 = lo;
    *t1 = hi;
    return hi > lo;
}

/* Source (V frame) and inverse 3x3 block of one view matrix. */
static int view_source(const double *P, double S[3], double Mi[9])
{
    const double a = P[0], b = P[1], c = P[2];
    const double d = P[4], e = P[5], f = P[6];
    const double g = P[8], h = P[9], i = P[10];
    double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
    double fro = 0.0;
    for (int k = 0; k < 12; ++k)
        if (k % 4 != 3)
            fro += P[k] * P[k];
    fro = sqrt(fro);
    if (!(fro > 0.0) || !(fabs(det) >= 1e-12 * fro * fro * fro))
        return OR_ESINGULAR;
    Mi[0] = (e * i - f * h) / det;
    Mi[1] = (c * h - b * i) / det;
    Mi[2] = (b * f - c * e) / det;
    Mi[3] = (f * g - d * i) / det;
    Mi[4] = (a * i - c * g) / det;
    Mi[5] = (c * d - a * f) / det;
    Mi[6] = (d * h - e * g) / det;
    Mi[7] = (b * g - a * h) / det;
    Mi[8] = (a * e - b * d) / det;
    for (int r = 0; r < 3; ++r)
        S[r] = -(Mi[3 * r] * P[3] + Mi[3 * r + 1] * P[7] + Mi[3 * r + 2] * P[11]);
    return OR_OK;
}

int oracle_forward_cyl(const double *P, int n_proj, int n_sub, int nu, int nv, int nr, int nphi,
                       int nz, double dr, double dz, const double *pose, double step,
                       const double *vol, const int *views, int n_views, double *out,
                       int64_t *count)
{
    cyl_t c;
    if (!views)
        n_views = n_proj;
    if (n_proj < 1 || n_sub < 1 || nu < 1 || nv < 1 || !(step > 0.0) || n_views < 0)
        return OR_EINVAL;
    if (cyl_init(&c, nr, nphi, nz, dr, dz, pose) != OR_OK)
        return OR_EINVAL;
    for (int k = 0; k < n_views; ++k)
        if (views && (views[k] < 0 || views[k] >= n_proj))
            return OR_EINVAL;
    /* set-up per sub-view, rejecting singular views and sources inside the hull */
    const size_t m = (size_t)n_proj * n_sub;
    double *Ss = malloc(sizeof(double) * 3 * m), *Ms = malloc(sizeof(double) * 9 * m);
    if (!Ss || !Ms) {
        free(Ss);
        free(Ms);
        return OR_EINVAL;
    }
    int st = OR_OK;
    for (size_t q = 0; q < m && st == OR_OK; ++q) {
        st = view_source(P + 12 * q, Ss + 3 * q, Ms + 9 * q);
        if (st == OR_OK) {
            double Sc[3];
            cyl_frame(&c, Ss + 3 * q, Sc);
            if (Sc[0] * Sc[0] + Sc[1] * Sc[1] <= cyl_rh(&c) * cyl_rh(&c) &&
                fabs(Sc[2]) <= cyl_hz(&c))
                st = OR_ESOURCE_INSIDE;
        }
    }
    if (st != OR_OK) {
        free(Ss);
        free(Ms);
        return st;
    }
    int64_t total = 0;
#pragma omp parallel for collapse(2) schedule(dynamic, 4) reduction(+ : total)
    for (int k = 0; k < n_views; ++k) {
        for (int iv = 0; iv < nv; ++iv) {
            int p = views ? views[k] : k;
            for (int iu = 0; iu < nu; ++iu) {
                double y = 0.0;
                for (int s = 0; s < n_sub; ++s) {
                    const size_t q = (size_t)p * n_sub + s;
                    const double *Mi = Ms + 9 * q;
                    double d[3], len = 0.0, Sc[3], dc[3], t0, t1;
                    for (int r = 0; r < 3; ++r) {
                        d[r] = Mi[3 * r] * iu + Mi[3 * r + 1] * iv + Mi[3 * r + 2];
                        len += d[r] * d[r];
                    }
                    len = sqrt(len);
                    for (int r = 0; r < 3; ++r)
                        d[r] /= len;
                    cyl_frame(&c, Ss + 3 * q, Sc);
                    for (int r = 0; r < 3; ++r)
                        dc[r] = c.R[3 * r] * d[0] + c.R[3 * r + 1] * d[1] + c.R[3 * r + 2] * d[2];
                    if (!cyl_clip(&c, Sc, dc, &t0, &t1))
                        continue;
                    double L = t1 - t0;
                    int n = (int)ceil(L / step);
                    if (n < 1)
                        n = 1;
                    double h = L / n, acc = 0.0;
                    for (int i = 0; i < n; ++i) {
                        double tt = t0 + (i + 0.5) * h, X[3];
                        for (int r = 0; r < 3; ++r)
                            X[r] = Sc[r] + tt * dc[r];
                        acc += cyl_value(&c, vol, X);
                    }
                    y += h * acc;
                    total += n;
                }
                out[((size_t)k * nv + iv) * nu + iu] = y / n_sub;
            }
        }
    }
    free(Ss);
    free(Ms);
    if (count)
        *count = total;
    return OR_OK;
}

int oracle_back_voxel_cyl(const double *P, int n_proj, int n_sub, int nu, int nv, int nr,
                          int nphi, int nz, double dr, double dz, const double *pose,
                          const double *sino, const int *views, int n_views, double *vol)
{
    cyl_t c;
    const double two_pi = 6.283185307179586476925287;
    if (!views)
        n_views = n_proj;
    if (cyl_init(&c, nr, nphi, nz, dr, dz, pose) != OR_OK)
        return OR_EINVAL;
    int st = check_voxel_args(n_proj, n_sub, nu, nv, nr, nphi, nz, views, n_views);
    if (st != OR_OK)
        return st;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < nphi; ++j)
            for (int i = 0; i < nr; ++i) {
                double r = (i + 0.5) * dr, phi = two_pi * j / nphi;
                double Xc[3] = {r * cos(phi), r * sin(phi), (k - 0.5 * (nz - 1)) * dz};
                double X[3];
                /* X = Rp^T (Xc - tp) */
                for (int q = 0; q < 3; ++q)
                    X[q] = c.R[q] * (Xc[0] - c.t[0]) + c.R[3 + q] * (Xc[1] - c.t[1]) +
                           c.R[6 + q] * (Xc[2] - c.t[2]);
                vol[((size_t)k * nphi + j) * nr + i] +=
                    voxel_sum(P, n_sub, nu, nv, sino, views, n_views, X[0], X[1], X[2]);
            }
    return OR_OK;
}
