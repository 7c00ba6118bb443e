/* Calls every exported function of the C oracle once on small inputs read
 * from a directory, and writes their outputs there as raw little-endian
 * float64 (counts as int64).  Built together with oracle/ctrex_oracle.c under
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitizers.py, which writes the inputs and compares the
 * outputs with the ordinary build of the oracle.
 *
 * Sizes (fixed here and in the test): 3 projections x 2 sub-views of 24 x 20
 * pixels; a 10 x 12 x 9 volume (x fastest); a 4 x 4 x 4 displacement grid; a
 * cylindrical grid of 6 rings x 16 angles x 9 slices (dr 1.5, dz 1).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_forward(const double *P, int n_proj, int n_sub, int nu, int nv, int nx, int ny,
                   int nz, double step, const double *vol, const int *views, int n_views,
                   const double *U, int gx, int gy, int gz, const double *tau, double *sino,
                   int64_t *n_samples);
int oracle_back(const double *P, int n_proj, int n_sub, int nu, int nv, int nx, int ny, int nz,
                double step, const double *sino, const int *views, int n_views, const double *U,
                int gx, int gy, int gz, const double *tau, double *vol);
int oracle_forward_indicator(const double *P, int n_proj, int n_sub, int nu, int nv, int nx,
                             int ny, int nz, double step, const double *Q, const double *centre,
                             double *sino);
int oracle_back_voxel(const double *P, int n_proj, int n_sub, int nu, int nv, int nx, int ny,
                      int nz, const double *sino, const int *views, int n_views, double *vol);
int oracle_back_voxel_points(const double *P, int n_proj, int n_sub, int nu, int nv, int nx,
                             int ny, int nz, const double *sino, const int *views, int n_views,
                             const int *ijk, int n_pts, double *out);
int oracle_forward_cyl(const double *P, int n_proj, int n_sub, int nu, int nv, int nr, int nphi,
                       int nz, double dr, double dz, const double *pose, double step,
                       const double *vol, const int *views, int n_views, double *out,
                       int64_t *count);
int oracle_back_voxel_cyl(const double *P, int n_proj, int n_sub, int nu, int nv, int nr,
                          int nphi, int nz, const double dr, double dz, const double *pose,
                          const double *sino, const int *views, int n_views, double *vol);

enum { NP = 3, NS = 2, NU = 24, NV = 20, NX = 10, NY = 12, NZ = 9, G = 4 };
enum { NR = 6, NPHI = 16, NZC = 9, NPTS = 5 };
#define NVOX (NX * NY * NZ)
#define NPIX (NP * NU * NV)
#define NCYL (NR * NPHI * NZC)

static const char *dir;

static void *load(const char *name, size_t bytes)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        exit(2);
    }
    void *p = malloc(bytes);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read %s\n", path);
        exit(2);
    }
    fclose(f);
    return p;
}

static void save(const char *name, const void *p, size_t bytes)
{
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot write %s\n", path);
        exit(2);
    }
    fclose(f);
}

static void check(int st, const char *what)
{
    if (st != 0) {
        fprintf(stderr, "%s returned %d\n", what, st);
        exit(3);
    }
}

int main(int argc, char **argv)
{
    if (argc != 2)
        return 2;
    dir = argv[1];
    double *P = load("P.bin", sizeof(double) * NP * NS * 12);
    double *vol = load("vol.bin", sizeof(double) * NVOX);
    double *sino = load("sino.bin", sizeof(double) * NPIX);
    double *U = load("U.bin", sizeof(double) * G * G * G * 3);
    double *tau = load("tau.bin", sizeof(double) * NP * NS);
    double *Q = load("Q.bin", sizeof(double) * 9);
    double *centre = load("centre.bin", sizeof(double) * 3);
    double *pose = load("pose.bin", sizeof(double) * 12);
    double *cvol = load("cvol.bin", sizeof(double) * NCYL);
    int *ijk = load("ijk.bin", sizeof(int) * 3 * NPTS);
    const int views[4] = {2, 0, 2, 1};

    double *y = calloc(NPIX, sizeof(double));
    double *y4 = calloc(4 * NU * NV, sizeof(double));
    double *x = calloc(NVOX, sizeof(double));
    double *c = calloc(NCYL, sizeof(double));
    double *pts = calloc(NPTS, sizeof(double));
    int64_t cnt[3] = {0, 0, 0};
    if (!y || !y4 || !x || !c || !pts)
        return 2;

    check(oracle_forward(P, NP, NS, NU, NV, NX, NY, NZ, 0.5, vol, NULL, NP, NULL, 0, 0, 0, NULL,
                         y, &cnt[0]), "forward");
    save("fwd.bin", y, sizeof(double) * NPIX);
    check(oracle_forward(P, NP, NS, NU, NV, NX, NY, NZ, 0.7, vol, views, 4, U, G, G, G, tau, y4,
                         &cnt[1]), "forward warp views");
    save("fwd_warp.bin", y4, sizeof(double) * 4 * NU * NV);
    check(oracle_back(P, NP, NS, NU, NV, NX, NY, NZ, 0.5, sino, NULL, NP, NULL, 0, 0, 0, NULL, x),
          "back");
    save("back.bin", x, sizeof(double) * NVOX);
    memset(x, 0, sizeof(double) * NVOX);
    check(oracle_back(P, NP, NS, NU, NV, NX, NY, NZ, 0.7, sino, views, 3, U, G, G,
                      G, tau, x), "back warp views");
    save("back_warp.bin", x, sizeof(double) * NVOX);
    check(oracle_forward_indicator(P, NP, NS, NU, NV, NX, NY, NZ, 0.5, Q, centre, y),
          "forward_indicator");
    save("indicator.bin", y, sizeof(double) * NPIX);
    memset(x, 0, sizeof(double) * NVOX);
    check(oracle_back_voxel(P, NP, NS, NU, NV, NX, NY, NZ, sino, NULL, NP, x), "back_voxel");
    save("back_voxel.bin", x, sizeof(double) * NVOX);
    check(oracle_back_voxel_points(P, NP, NS, NU, NV, NX, NY, NZ, sino, views, 3, ijk, NPTS, pts),
          "back_voxel_points");
    save("points.bin", pts, sizeof(double) * NPTS);
    check(oracle_forward_cyl(P, NP, NS, NU, NV, NR, NPHI, NZC, 1.5, 1.0, pose, 0.5, cvol, NULL, NP,
                             y, &cnt[2]), "forward_cyl");
    save("fwd_cyl.bin", y, sizeof(double) * NPIX);
    check(oracle_back_voxel_cyl(P, NP, NS, NU, NV, NR, NPHI, NZC, 1.5, 1.0, pose, sino, NULL, NP,
                                c), "back_voxel_cyl");
    save("back_cyl.bin", c, sizeof(double) * NCYL);
    save("counts.bin", cnt, sizeof cnt);

    free(P), free(vol), free(sino), free(U), free(tau), free(Q), free(centre), free(pose);
    free(cvol), free(ijk), free(y), free(y4), free(x), free(c), free(pts);
    puts("ok");
    return 0;
}
