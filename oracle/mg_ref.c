/*
 * ORACLE -- test infrastructure, not the product.
 *
 * Plain, slow FP64 multigrid for the two scalar elliptic problems of the
 * NR99 linear magnetohydrostatic model, written from Section 2.2 of
 * MacTaggart et al., "Non-symmetric magnetohydrostatic equilibria: a
 * multigrid approach":
 *
 *   lower boundary, equation (11):
 *       P_xx + P_yy = -Bz(x, y),   P = 0 on the edges of the base;
 *   interior, equation (8):
 *       (1 - xi(z)) (P_xx + P_yy) + P_zz + alpha^2 P = 0,
 *       with P(z = 0) taken from (11) and P = 0 on the top and side faces
 *       (the B = 0 walls of Section 2.2).
 *
 * Both are discretised with second-order central differences on a uniform
 * vertex-centred grid of n = 2^L + 1 nodes per axis, x fastest:
 * idx = i + nx*(j + ny*k).  The multigrid method (Section 2.2, the solver
 * stages named in Section 4: relaxation, residual, reduction, prolongation)
 * is a V(nu1, nu2) cycle with
 *   - red-black Gauss-Seidel relaxation, red = (i+j+k) even, red first;
 *   - full-weighting restriction (27-point in 3D, 9-point in 2D) of the
 *     residual, which is zero on boundary nodes;
 *   - trilinear (bilinear) prolongation of the coarse correction;
 *   - coarse operators by rediscretisation with doubled spacing and xi
 *     sampled at the coarse nodes;
 *   - coarsening of every axis, except that a step keeps z when the z
 *     spacing is at least sqrt(2) times the larger in-plane spacing (x-y
 *     semicoarsening: residual weighted and correction interpolated within
 *     each plane) and keeps x and y when the z spacing is at most 1/sqrt(2)
 *     times the smaller in-plane spacing (z semicoarsening: weighting and
 *     interpolation along z only), while every axis that is halved has more
 *     than 3 nodes, and an exact dense solve (Gaussian elimination with
 *     partial pivoting) on the coarsest grid.  The paper does not say how
 *     the coarse grids are built; this rule brings the coarse levels of
 *     grids with dz != dx toward equal spacing, which point relaxation
 *     needs to smooth in every direction.
 * Stopping rule: ||r_k||_2 / ||r_0||_2 <= rtol over interior nodes, with
 * r_0 the residual of the initial iterate (P = 0 in the interior, step 1 of
 * the procedure in Section 2.2).
 *
 * The last section solves the general scalar problem Section 2.2 reduces
 * the model to, a(x) lap u + b(x) u = c(x) with u given on the boundary, in
 * the box or on one of its faces, by the same multigrid (ref_gen_*).
 *
 * Each function below is a direct loop over the definition it cites; there
 * is no blocking or fusion.  OpenMP pragmas (when built with -fopenmp)
 * split the outer loop of the 3D residual, of each colour of a sweep and of
 * the grid transfers over threads, for timing only: every node's value is
 * computed as in the serial loop and no sum is split, so the results do not
 * depend on the number of threads.  Only tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code with
 * the HIP path.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_OK 0
#define REF_NO_CONVERGENCE 1
#define REF_DIVERGED 2
#define REF_BAD_GRID (-1)
#define REF_SINGULAR (-2)
#define REF_NOMEM (-3)

#define AT3(a, i, j, k) (a)[(size_t)(i) + (size_t)nx * ((size_t)(j) + (size_t)ny * (size_t)(k))]
#define AT2(a, i, j) (a)[(size_t)(i) + (size_t)nx * (size_t)(j)]

/* Threads the parallel loops use (n >= 1); returns the count in effect
 * (1 without OpenMP). */
int ref_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* grid hierarchy                                                       */
/* ------------------------------------------------------------------ */

static int valid_axis(int n)
{
    if (n < 3) return 0;
    int m = n - 1;
    return (m & (m - 1)) == 0;
}

/* Kind of the step from a grid of n nodes on a box of lengths len:
 * STEP_XY (z kept) when dz^2 >= 2 max(dx, dy)^2, STEP_Z (x and y kept) when
 * 2 dz^2 <= min(dx, dy)^2, else STEP_ALL. */
#define STEP_ALL 0
#define STEP_XY 1
#define STEP_Z 2
static int step_kind(const int *n, const double *len)
{
    double hx = len[0] / (double)(n[0] - 1), hy = len[1] / (double)(n[1] - 1);
    double hz = len[2] / (double)(n[2] - 1);
    double hmax = hx > hy ? hx : hy, hmin = hx < hy ? hx : hy;
    if (hz * hz >= 2.0 * hmax * hmax) return STEP_XY;
    if (2.0 * hz * hz <= hmin * hmin) return STEP_Z;
    return STEP_ALL;
}

/* Number of levels of the 3D hierarchy; kinds (may be NULL, room for 32
 * entries) receives the kind of each step l -> l+1 (STEP_ALL: every axis
 * halved, STEP_XY: x and y halved, STEP_Z: z halved).  Coarsening stops
 * when an axis that the next step would halve has 3 nodes. */
int ref_levels3(const int *n0, const double *len, int *kinds)
{
    if (!valid_axis(n0[0]) || !valid_axis(n0[1]) || !valid_axis(n0[2])) return REF_BAD_GRID;
    int n[3] = {n0[0], n0[1], n0[2]};
    int L = 1;
    for (;;) {
        int kind = step_kind(n, len);
        int hxy = kind != STEP_Z, hz = kind != STEP_XY;
        if ((hxy && (n[0] <= 3 || n[1] <= 3)) || (hz && n[2] <= 3)) break;
        if (kinds && L - 1 < 32) kinds[L - 1] = kind;
        if (hxy) {
            n[0] = (n[0] - 1) / 2 + 1;
            n[1] = (n[1] - 1) / 2 + 1;
        }
        if (hz) n[2] = (n[2] - 1) / 2 + 1;
        L++;
    }
    return L;
}

int ref_nlevels2(int nx, int ny)
{
    if (!valid_axis(nx) || !valid_axis(ny)) return REF_BAD_GRID;
    int L = 1;
    while (nx > 3 && ny > 3) {
        nx = (nx - 1) / 2 + 1;
        ny = (ny - 1) / 2 + 1;
        L++;
    }
    return L;
}

/* ------------------------------------------------------------------ */
/* 3D operator of equation (8)                                          */
/* ------------------------------------------------------------------ */

/* (A u) at an interior node: (1-xi_k)(d2x u + d2y u) + d2z u + alpha^2 u. */
static double op3_at(const double *u, int nx, int ny, int i, int j, int k,
                     double dx, double dy, double dz, double xik, double alpha)
{
    double c = AT3(u, i, j, k);
    double uxx = (AT3(u, i + 1, j, k) - 2.0 * c + AT3(u, i - 1, j, k)) / (dx * dx);
    double uyy = (AT3(u, i, j + 1, k) - 2.0 * c + AT3(u, i, j - 1, k)) / (dy * dy);
    double uzz = (AT3(u, i, j, k + 1) - 2.0 * c + AT3(u, i, j, k - 1)) / (dz * dz);
    return (1.0 - xik) * (uxx + uyy) + uzz + alpha * alpha * c;
}

/* r = f - A u on interior nodes, r = 0 on boundary nodes; f may be NULL (0). */
void ref_residual3(const int *n, const double *h, const double *xi, double alpha,
                   const double *u, const double *f, double *r)
{
    int nx = n[0], ny = n[1], nz = n[2];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double v = 0.0;
                if (i > 0 && i < nx - 1 && j > 0 && j < ny - 1 && k > 0 && k < nz - 1) {
                    double fv = f ? AT3(f, i, j, k) : 0.0;
                    v = fv - op3_at(u, nx, ny, i, j, k, h[0], h[1], h[2], xi[k], alpha);
                }
                AT3(r, i, j, k) = v;
            }
}

double ref_norm3_interior(const int *n, const double *r)
{
    int nx = n[0], ny = n[1], nz = n[2];
    double s = 0.0;
    for (int k = 1; k < nz - 1; k++)
        for (int j = 1; j < ny - 1; j++)
            for (int i = 1; i < nx - 1; i++) s += AT3(r, i, j, k) * AT3(r, i, j, k);
    return sqrt(s);
}

/* One Gauss-Seidel update of node (i,j,k): solve its row of A u = f for u. */
static void gs3_point(double *u, const double *f, int nx, int ny, int i, int j, int k,
                      double dx, double dy, double dz, double xik, double alpha)
{
    double ax = (1.0 - xik) / (dx * dx);
    double ay = (1.0 - xik) / (dy * dy);
    double az = 1.0 / (dz * dz);
    double diag = alpha * alpha - 2.0 * ax - 2.0 * ay - 2.0 * az;
    double off = ax * (AT3(u, i + 1, j, k) + AT3(u, i - 1, j, k)) +
                 ay * (AT3(u, i, j + 1, k) + AT3(u, i, j - 1, k)) +
                 az * (AT3(u, i, j, k + 1) + AT3(u, i, j, k - 1));
    double fv = f ? AT3(f, i, j, k) : 0.0;
    AT3(u, i, j, k) = (fv - off) / diag;
}

/* nsweeps red-black Gauss-Seidel sweeps in place: all red nodes
 * ((i+j+k) even) first, then all black nodes. */
void ref_rbgs3(const int *n, const double *h, const double *xi, double alpha,
               double *u, const double *f, int nsweeps)
{
    int nx = n[0], ny = n[1], nz = n[2];
    for (int s = 0; s < nsweeps; s++)
        for (int colour = 0; colour < 2; colour++) {
            /* nodes of one colour read only the other colour */
#pragma omp parallel for schedule(static)
            for (int k = 1; k < nz - 1; k++)
                for (int j = 1; j < ny - 1; j++)
                    for (int i = 1; i < nx - 1; i++)
                        if (((i + j + k) & 1) == colour)
                            gs3_point(u, f, nx, ny, i, j, k, h[0], h[1], h[2], xi[k], alpha);
        }
}

/* Full weighting: fc(I,J,K) = sum w(a)w(b)w(c) rf(2I+a, 2J+b, 2K+c) with
 * w(0) = 1/2, w(+-1) = 1/4, at coarse interior nodes; coarse boundary = 0. */
void ref_restrict3(const int *nf, const double *rf, double *fc)
{
    static const double w[3] = {0.25, 0.5, 0.25};
    int nxf = nf[0], nyf = nf[1];
    int ncx = (nf[0] - 1) / 2 + 1, ncy = (nf[1] - 1) / 2 + 1, ncz = (nf[2] - 1) / 2 + 1;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < ncz; K++)
        for (int J = 0; J < ncy; J++)
            for (int I = 0; I < ncx; I++) {
                double s = 0.0;
                if (I > 0 && I < ncx - 1 && J > 0 && J < ncy - 1 && K > 0 && K < ncz - 1) {
                    for (int c = -1; c <= 1; c++)
                        for (int b = -1; b <= 1; b++)
                            for (int a = -1; a <= 1; a++) {
                                size_t idx = (size_t)(2 * I + a) +
                                             (size_t)nxf * ((size_t)(2 * J + b) + (size_t)nyf * (size_t)(2 * K + c));
                                s += w[a + 1] * w[b + 1] * w[c + 1] * rf[idx];
                            }
                }
                fc[(size_t)I + (size_t)ncx * ((size_t)J + (size_t)ncy * (size_t)K)] = s;
            }
}

/* Full weighting within each plane (z kept): fc(I,J,k) = sum w(a)w(b)
 * rf(2I+a, 2J+b, k), at coarse interior nodes; coarse boundary = 0. */
void ref_restrict3_xy(const int *nf, const double *rf, double *fc)
{
    static const double w[3] = {0.25, 0.5, 0.25};
    int nxf = nf[0], nyf = nf[1], nz = nf[2];
    int ncx = (nf[0] - 1) / 2 + 1, ncy = (nf[1] - 1) / 2 + 1;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int J = 0; J < ncy; J++)
            for (int I = 0; I < ncx; I++) {
                double s = 0.0;
                if (I > 0 && I < ncx - 1 && J > 0 && J < ncy - 1 && k > 0 && k < nz - 1) {
                    for (int b = -1; b <= 1; b++)
                        for (int a = -1; a <= 1; a++) {
                            size_t idx = (size_t)(2 * I + a) +
                                         (size_t)nxf * ((size_t)(2 * J + b) + (size_t)nyf * (size_t)k);
                            s += w[a + 1] * w[b + 1] * rf[idx];
                        }
                }
                fc[(size_t)I + (size_t)ncx * ((size_t)J + (size_t)ncy * (size_t)k)] = s;
            }
}

/* Linear interpolation weight of coarse node C for fine index i along one
 * axis: 1 if i == 2C, 1/2 if |i - 2C| == 1, else 0. */
static double lin_w(int i, int C)
{
    int d = i - 2 * C;
    if (d == 0) return 1.0;
    if (d == 1 || d == -1) return 0.5;
    return 0.0;
}

/* uf += I(ec) on fine interior nodes, I = trilinear interpolation. */
void ref_prolong3(const int *nc, const double *ec, double *uf)
{
    int ncx = nc[0], ncy = nc[1], ncz = nc[2];
    int nx = 2 * (ncx - 1) + 1, ny = 2 * (ncy - 1) + 1, nz = 2 * (ncz - 1) + 1;
#pragma omp parallel for schedule(static)
    for (int k = 1; k < nz - 1; k++)
        for (int j = 1; j < ny - 1; j++)
            for (int i = 1; i < nx - 1; i++) {
                double s = 0.0;
                for (int K = k / 2; K <= (k + 1) / 2; K++)
                    for (int J = j / 2; J <= (j + 1) / 2; J++)
                        for (int I = i / 2; I <= (i + 1) / 2; I++)
                            s += lin_w(i, I) * lin_w(j, J) * lin_w(k, K) *
                                 ec[(size_t)I + (size_t)ncx * ((size_t)J + (size_t)ncy * (size_t)K)];
                AT3(uf, i, j, k) += s;
            }
}

/* Full weighting along z (x and y kept): fc(i,j,K) = sum w(c) rf(i, j, 2K+c)
 * at coarse interior nodes; coarse boundary = 0. */
void ref_restrict3_z(const int *nf, const double *rf, double *fc)
{
    static const double w[3] = {0.25, 0.5, 0.25};
    int nx = nf[0], ny = nf[1];
    int ncz = (nf[2] - 1) / 2 + 1;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < ncz; K++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double s = 0.0;
                if (i > 0 && i < nx - 1 && j > 0 && j < ny - 1 && K > 0 && K < ncz - 1)
                    for (int c = -1; c <= 1; c++) s += w[c + 1] * AT3(rf, i, j, 2 * K + c);
                AT3(fc, i, j, K) = s;
            }
}

/* uf += I(ec) on fine interior nodes, I = linear interpolation along z
 * (x and y kept). */
void ref_prolong3_z(const int *nc, const double *ec, double *uf)
{
    int nx = nc[0], ny = nc[1], ncz = nc[2];
    int nz = 2 * (ncz - 1) + 1;
#pragma omp parallel for schedule(static)
    for (int k = 1; k < nz - 1; k++)
        for (int j = 1; j < ny - 1; j++)
            for (int i = 1; i < nx - 1; i++) {
                double s = 0.0;
                for (int K = k / 2; K <= (k + 1) / 2; K++) s += lin_w(k, K) * AT3(ec, i, j, K);
                AT3(uf, i, j, k) += s;
            }
}

/* uf += I(ec) on fine interior nodes, I = bilinear interpolation within
 * each plane (z kept). */
void ref_prolong3_xy(const int *nc, const double *ec, double *uf)
{
    int ncx = nc[0], ncy = nc[1], nz = nc[2];
    int nx = 2 * (ncx - 1) + 1, ny = 2 * (ncy - 1) + 1;
#pragma omp parallel for schedule(static)
    for (int k = 1; k < nz - 1; k++)
        for (int j = 1; j < ny - 1; j++)
            for (int i = 1; i < nx - 1; i++) {
                double s = 0.0;
                for (int J = j / 2; J <= (j + 1) / 2; J++)
                    for (int I = i / 2; I <= (i + 1) / 2; I++)
                        s += lin_w(i, I) * lin_w(j, J) *
                             ec[(size_t)I + (size_t)ncx * ((size_t)J + (size_t)ncy * (size_t)k)];
                AT3(uf, i, j, k) += s;
            }
}

/* ------------------------------------------------------------------ */
/* dense direct solve of the interior unknowns                          */
/* ------------------------------------------------------------------ */

/* Solve M x = b (m unknowns, row-major M), Gaussian elimination with
 * partial pivoting.  M and b are overwritten. */
static int gauss_solve(double *M, double *b, double *x, int m)
{
    for (int c = 0; c < m; c++) {
        int p = c;
        for (int r = c + 1; r < m; r++)
            if (fabs(M[(size_t)r * m + c]) > fabs(M[(size_t)p * m + c])) p = r;
        if (M[(size_t)p * m + c] == 0.0) return REF_SINGULAR;
        if (p != c) {
            for (int q = 0; q < m; q++) {
                double t = M[(size_t)c * m + q];
                M[(size_t)c * m + q] = M[(size_t)p * m + q];
                M[(size_t)p * m + q] = t;
            }
            double t = b[c];
            b[c] = b[p];
            b[p] = t;
        }
        for (int r = c + 1; r < m; r++) {
            double l = M[(size_t)r * m + c] / M[(size_t)c * m + c];
            if (l == 0.0) continue;
            for (int q = c; q < m; q++) M[(size_t)r * m + q] -= l * M[(size_t)c * m + q];
            b[r] -= l * b[c];
        }
    }
    for (int r = m - 1; r >= 0; r--) {
        double s = b[r];
        for (int q = r + 1; q < m; q++) s -= M[(size_t)r * m + q] * x[q];
        x[r] = s / M[(size_t)r * m + r];
    }
    return REF_OK;
}

/* Exact solve of A u = f for the interior nodes of one 3D grid; boundary
 * values are taken from u and moved to the right-hand side. */
int ref_direct3(const int *n, const double *h, const double *xi, double alpha,
                double *u, const double *f)
{
    int nx = n[0], ny = n[1], nz = n[2];
    int mx = nx - 2, my = ny - 2, mz = nz - 2;
    int m = mx * my * mz;
    double *M = (double *)calloc((size_t)m * m, sizeof(double));
    double *b = (double *)calloc((size_t)m, sizeof(double));
    double *x = (double *)calloc((size_t)m, sizeof(double));
    if (!M || !b || !x) {
        free(M); free(b); free(x);
        return REF_NOMEM;
    }
    double dx = h[0], dy = h[1], dz = h[2];
    for (int k = 1; k < nz - 1; k++)
        for (int j = 1; j < ny - 1; j++)
            for (int i = 1; i < nx - 1; i++) {
                int row = (i - 1) + mx * ((j - 1) + my * (k - 1));
                double ax = (1.0 - xi[k]) / (dx * dx), ay = (1.0 - xi[k]) / (dy * dy), az = 1.0 / (dz * dz);
                double rhs = f ? AT3(f, i, j, k) : 0.0;
                M[(size_t)row * m + row] = alpha * alpha - 2.0 * ax - 2.0 * ay - 2.0 * az;
                int nb[6][3] = {{i + 1, j, k}, {i - 1, j, k}, {i, j + 1, k}, {i, j - 1, k}, {i, j, k + 1}, {i, j, k - 1}};
                double cf[6] = {ax, ax, ay, ay, az, az};
                for (int q = 0; q < 6; q++) {
                    int a = nb[q][0], bb = nb[q][1], c = nb[q][2];
                    if (a == 0 || a == nx - 1 || bb == 0 || bb == ny - 1 || c == 0 || c == nz - 1)
                        rhs -= cf[q] * AT3(u, a, bb, c);
                    else
                        M[(size_t)row * m + ((a - 1) + mx * ((bb - 1) + my * (c - 1)))] += cf[q];
                }
                b[row] = rhs;
            }
    int st = gauss_solve(M, b, x, m);
    if (st == REF_OK)
        for (int k = 1; k < nz - 1; k++)
            for (int j = 1; j < ny - 1; j++)
                for (int i = 1; i < nx - 1; i++)
                    AT3(u, i, j, k) = x[(i - 1) + mx * ((j - 1) + my * (k - 1))];
    free(M); free(b); free(x);
    return st;
}

/* ------------------------------------------------------------------ */
/* 3D V-cycle and solve                                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    int n[3];
    double h[3];
    double *xi; /* xi sampled at this level's z nodes */
    double *u, *f, *r;
    size_t N;
    int kind;   /* kind of the step to the next level (STEP_*) */
} lev3;

static void free_levels3(lev3 *lv, int L)
{
    for (int l = 0; l < L; l++) {
        free(lv[l].xi);
        if (l > 0) { free(lv[l].u); free(lv[l].f); }
        free(lv[l].r);
    }
}

static int build_levels3(lev3 *lv, int L, const int *n, const double *len, const double *xi,
                         double *u0, const double *f0)
{
    memset(lv, 0, sizeof(lev3) * (size_t)L);
    int kinds[32] = {0};
    if (ref_levels3(n, len, kinds) != L) return REF_BAD_GRID;
    int nn[3] = {n[0], n[1], n[2]};
    size_t stride = 1; /* fine z nodes per z step of this level */
    for (int l = 0; l < L; l++) {
        for (int a = 0; a < 3; a++) {
            lv[l].n[a] = nn[a];
            lv[l].h[a] = len[a] / (double)(nn[a] - 1);
        }
        lv[l].N = (size_t)nn[0] * nn[1] * nn[2];
        lv[l].xi = (double *)malloc(sizeof(double) * (size_t)nn[2]);
        lv[l].r = (double *)calloc(lv[l].N, sizeof(double));
        if (!lv[l].xi || !lv[l].r) return REF_NOMEM;
        for (int k = 0; k < nn[2]; k++) lv[l].xi[k] = xi[(size_t)k * stride];
        lv[l].kind = (l < L - 1) ? kinds[l] : STEP_ALL;
        if (l == 0) {
            lv[l].u = u0;
            lv[l].f = (double *)f0;
        } else {
            lv[l].u = (double *)calloc(lv[l].N, sizeof(double));
            lv[l].f = (double *)calloc(lv[l].N, sizeof(double));
            if (!lv[l].u || !lv[l].f) return REF_NOMEM;
        }
        if (lv[l].kind != STEP_Z) {
            nn[0] = (nn[0] - 1) / 2 + 1;
            nn[1] = (nn[1] - 1) / 2 + 1;
        }
        if (lv[l].kind != STEP_XY) {
            nn[2] = (nn[2] - 1) / 2 + 1;
            stride *= 2;
        }
    }
    return REF_OK;
}

static int vcycle3(lev3 *lv, int l, int L, double alpha, int nu1, int nu2)
{
    lev3 *c = &lv[l];
    if (l == L - 1) return ref_direct3(c->n, c->h, c->xi, alpha, c->u, c->f);
    ref_rbgs3(c->n, c->h, c->xi, alpha, c->u, c->f, nu1);
    ref_residual3(c->n, c->h, c->xi, alpha, c->u, c->f, c->r);
    lev3 *d = &lv[l + 1];
    if (c->kind == STEP_XY)
        ref_restrict3_xy(c->n, c->r, d->f);
    else if (c->kind == STEP_Z)
        ref_restrict3_z(c->n, c->r, d->f);
    else
        ref_restrict3(c->n, c->r, d->f);
    memset(d->u, 0, sizeof(double) * d->N);
    int st = vcycle3(lv, l + 1, L, alpha, nu1, nu2);
    if (st != REF_OK) return st;
    if (c->kind == STEP_XY)
        ref_prolong3_xy(d->n, d->u, c->u);
    else if (c->kind == STEP_Z)
        ref_prolong3_z(d->n, d->u, c->u);
    else
        ref_prolong3(d->n, d->u, c->u);
    ref_rbgs3(c->n, c->h, c->xi, alpha, c->u, c->f, nu2);
    return REF_OK;
}

/* Multigrid solve of equation (8) for P (nx*ny*nz, x fastest) in place.
 * P's boundary values are the Dirichlet data (plane k=0 from the lower
 * boundary solve, zero elsewhere); interior values are the initial guess.
 * len = (lx, ly, lz).  Runs V(nu1,nu2) cycles until ||r||/||r0|| <= rtol or
 * max_cycles.  hist (may be NULL) receives ||r_c|| for c = 0..cycles. */
int ref_mg3(const int *n, const double *len, const double *xi, double alpha, double *P,
            double rtol, int max_cycles, int nu1, int nu2, int *cycles_out,
            double *relres_out, double *hist)
{
    int L = ref_levels3(n, len, NULL);
    if (L < 1) return REF_BAD_GRID;
    lev3 *lv = (lev3 *)calloc((size_t)L, sizeof(lev3));
    if (!lv) return REF_NOMEM;
    int st = build_levels3(lv, L, n, len, xi, P, NULL);
    if (st != REF_OK) { free_levels3(lv, L); free(lv); return st; }

    ref_residual3(lv[0].n, lv[0].h, lv[0].xi, alpha, P, NULL, lv[0].r);
    double r0 = ref_norm3_interior(lv[0].n, lv[0].r);
    double res = r0;
    if (hist) hist[0] = r0;
    int cycles = 0;
    st = REF_NO_CONVERGENCE;
    if (r0 == 0.0) st = REF_OK;
    while (st == REF_NO_CONVERGENCE && cycles < max_cycles) {
        int s2 = vcycle3(lv, 0, L, alpha, nu1, nu2);
        if (s2 != REF_OK) { st = s2; break; }
        cycles++;
        ref_residual3(lv[0].n, lv[0].h, lv[0].xi, alpha, P, NULL, lv[0].r);
        res = ref_norm3_interior(lv[0].n, lv[0].r);
        if (hist) hist[cycles] = res;
        if (!isfinite(res) || res > 10.0 * r0) { st = REF_DIVERGED; break; }
        if (res <= rtol * r0) st = REF_OK;
    }
    if (cycles_out) *cycles_out = cycles;
    if (relres_out) *relres_out = (r0 > 0.0) ? res / r0 : 0.0;
    free_levels3(lv, L);
    free(lv);
    return st;
}

/* One V-cycle at the finest level of an arbitrary problem A u = f (f may be
 * NULL): exposes the cycle itself for iterate-by-iterate comparisons. */
int ref_vcycle3_once(const int *n, const double *len, const double *xi, double alpha,
                     double *u, const double *f, int nu1, int nu2)
{
    int L = ref_levels3(n, len, NULL);
    if (L < 1) return REF_BAD_GRID;
    lev3 *lv = (lev3 *)calloc((size_t)L, sizeof(lev3));
    if (!lv) return REF_NOMEM;
    int st = build_levels3(lv, L, n, len, xi, u, f);
    if (st == REF_OK) st = vcycle3(lv, 0, L, alpha, nu1, nu2);
    free_levels3(lv, L);
    free(lv);
    return st;
}

/* ------------------------------------------------------------------ */
/* 2D problem, equation (11): (d2x + d2y) P = -Bz, P = 0 on the edges   */
/* ------------------------------------------------------------------ */

static double op2_at(const double *u, int nx, int i, int j, double dx, double dy)
{
    double c = AT2(u, i, j);
    return (AT2(u, i + 1, j) - 2.0 * c + AT2(u, i - 1, j)) / (dx * dx) +
           (AT2(u, i, j + 1) - 2.0 * c + AT2(u, i, j - 1)) / (dy * dy);
}

void ref_residual2(const int *n, const double *h, const double *u, const double *f, double *r)
{
    int nx = n[0], ny = n[1];
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            double v = 0.0;
            if (i > 0 && i < nx - 1 && j > 0 && j < ny - 1)
                v = (f ? AT2(f, i, j) : 0.0) - op2_at(u, nx, i, j, h[0], h[1]);
            AT2(r, i, j) = v;
        }
}

double ref_norm2_interior(const int *n, const double *r)
{
    int nx = n[0], ny = n[1];
    double s = 0.0;
    for (int j = 1; j < ny - 1; j++)
        for (int i = 1; i < nx - 1; i++) s += AT2(r, i, j) * AT2(r, i, j);
    return sqrt(s);
}

void ref_rbgs2(const int *n, const double *h, double *u, const double *f, int nsweeps)
{
    int nx = n[0], ny = n[1];
    double ax = 1.0 / (h[0] * h[0]), ay = 1.0 / (h[1] * h[1]);
    double diag = -2.0 * ax - 2.0 * ay;
    for (int s = 0; s < nsweeps; s++)
        for (int colour = 0; colour < 2; colour++)
            for (int j = 1; j < ny - 1; j++)
                for (int i = 1; i < nx - 1; i++)
                    if (((i + j) & 1) == colour) {
                        double off = ax * (AT2(u, i + 1, j) + AT2(u, i - 1, j)) +
                                     ay * (AT2(u, i, j + 1) + AT2(u, i, j - 1));
                        AT2(u, i, j) = ((f ? AT2(f, i, j) : 0.0) - off) / diag;
                    }
}

void ref_restrict2(const int *nf, const double *rf, double *fc)
{
    static const double w[3] = {0.25, 0.5, 0.25};
    int nxf = nf[0];
    int ncx = (nf[0] - 1) / 2 + 1, ncy = (nf[1] - 1) / 2 + 1;
    for (int J = 0; J < ncy; J++)
        for (int I = 0; I < ncx; I++) {
            double s = 0.0;
            if (I > 0 && I < ncx - 1 && J > 0 && J < ncy - 1)
                for (int b = -1; b <= 1; b++)
                    for (int a = -1; a <= 1; a++)
                        s += w[a + 1] * w[b + 1] * rf[(size_t)(2 * I + a) + (size_t)nxf * (size_t)(2 * J + b)];
            fc[(size_t)I + (size_t)ncx * (size_t)J] = s;
        }
}

void ref_prolong2(const int *nc, const double *ec, double *uf)
{
    int ncx = nc[0], ncy = nc[1];
    int nx = 2 * (ncx - 1) + 1, ny = 2 * (ncy - 1) + 1;
    for (int j = 1; j < ny - 1; j++)
        for (int i = 1; i < nx - 1; i++) {
            double s = 0.0;
            for (int J = j / 2; J <= (j + 1) / 2; J++)
                for (int I = i / 2; I <= (i + 1) / 2; I++)
                    s += lin_w(i, I) * lin_w(j, J) * ec[(size_t)I + (size_t)ncx * (size_t)J];
            AT2(uf, i, j) += s;
        }
    (void)ny;
}

int ref_direct2(const int *n, const double *h, double *u, const double *f)
{
    int nx = n[0], ny = n[1];
    int mx = nx - 2, my = ny - 2, m = mx * my;
    double *M = (double *)calloc((size_t)m * m, sizeof(double));
    double *b = (double *)calloc((size_t)m, sizeof(double));
    double *x = (double *)calloc((size_t)m, sizeof(double));
    if (!M || !b || !x) {
        free(M); free(b); free(x);
        return REF_NOMEM;
    }
    double ax = 1.0 / (h[0] * h[0]), ay = 1.0 / (h[1] * h[1]);
    for (int j = 1; j < ny - 1; j++)
        for (int i = 1; i < nx - 1; i++) {
            int row = (i - 1) + mx * (j - 1);
            double rhs = f ? AT2(f, i, j) : 0.0;
            M[(size_t)row * m + row] = -2.0 * ax - 2.0 * ay;
            int nb[4][2] = {{i + 1, j}, {i - 1, j}, {i, j + 1}, {i, j - 1}};
            double cf[4] = {ax, ax, ay, ay};
            for (int q = 0; q < 4; q++) {
                int a = nb[q][0], bb = nb[q][1];
                if (a == 0 || a == nx - 1 || bb == 0 || bb == ny - 1)
                    rhs -= cf[q] * AT2(u, a, bb);
                else
                    M[(size_t)row * m + ((a - 1) + mx * (bb - 1))] += cf[q];
            }
            b[row] = rhs;
        }
    int st = gauss_solve(M, b, x, m);
    if (st == REF_OK)
        for (int j = 1; j < ny - 1; j++)
            for (int i = 1; i < nx - 1; i++) AT2(u, i, j) = x[(i - 1) + mx * (j - 1)];
    free(M); free(b); free(x);
    return st;
}

typedef struct {
    int n[2];
    double h[2];
    double *u, *f, *r;
    size_t N;
} lev2;

static int vcycle2(lev2 *lv, int l, int L, int nu1, int nu2)
{
    lev2 *c = &lv[l];
    if (l == L - 1) return ref_direct2(c->n, c->h, c->u, c->f);
    ref_rbgs2(c->n, c->h, c->u, c->f, nu1);
    ref_residual2(c->n, c->h, c->u, c->f, c->r);
    lev2 *d = &lv[l + 1];
    ref_restrict2(c->n, c->r, d->f);
    memset(d->u, 0, sizeof(double) * d->N);
    int st = vcycle2(lv, l + 1, L, nu1, nu2);
    if (st != REF_OK) return st;
    ref_prolong2(d->n, d->u, c->u);
    ref_rbgs2(c->n, c->h, c->u, c->f, nu2);
    return REF_OK;
}

/* Multigrid solve of equation (11) on the lower boundary: P0 (nx*ny, x
 * fastest) receives the solution; its interior is the initial guess.  Its
 * edges are set to zero (the B = 0 side walls of Section 2.2), or, with
 * keep_edges, kept as the Dirichlet data (the summary of Section 5 leaves
 * P on the side boundaries to the problem).  Bz0 on edge nodes is not
 * read. */
int ref_mg2_edges(const int *n, const double *len, const double *bz0, double *P0, double rtol,
                  int max_cycles, int nu1, int nu2, int *cycles_out, double *relres_out, double *hist,
                  int keep_edges)
{
    int L = ref_nlevels2(n[0], n[1]);
    if (L < 1) return REF_BAD_GRID;
    int nx = n[0], ny = n[1];
    lev2 *lv = (lev2 *)calloc((size_t)L, sizeof(lev2));
    if (!lv) return REF_NOMEM;
    int nn[2] = {n[0], n[1]};
    int st = REF_OK;
    for (int l = 0; l < L; l++) {
        lv[l].n[0] = nn[0];
        lv[l].n[1] = nn[1];
        lv[l].h[0] = len[0] / (double)(nn[0] - 1);
        lv[l].h[1] = len[1] / (double)(nn[1] - 1);
        lv[l].N = (size_t)nn[0] * nn[1];
        lv[l].u = (l == 0) ? P0 : (double *)calloc(lv[l].N, sizeof(double));
        lv[l].f = (double *)calloc(lv[l].N, sizeof(double));
        lv[l].r = (double *)calloc(lv[l].N, sizeof(double));
        if (!lv[l].u || !lv[l].f || !lv[l].r) st = REF_NOMEM;
        nn[0] = (nn[0] - 1) / 2 + 1;
        nn[1] = (nn[1] - 1) / 2 + 1;
    }
    double r0 = 0.0, res = 0.0;
    int cycles = 0;
    if (st == REF_OK) {
        /* right-hand side of (11) on interior nodes; P = 0 on the edges */
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int edge = (i == 0 || i == nx - 1 || j == 0 || j == ny - 1);
                AT2(lv[0].f, i, j) = edge ? 0.0 : -AT2(bz0, i, j);
                if (edge && !keep_edges) AT2(P0, i, j) = 0.0;
            }
        ref_residual2(lv[0].n, lv[0].h, P0, lv[0].f, lv[0].r);
        r0 = ref_norm2_interior(lv[0].n, lv[0].r);
        res = r0;
        if (hist) hist[0] = r0;
        st = (r0 == 0.0) ? REF_OK : REF_NO_CONVERGENCE;
        while (st == REF_NO_CONVERGENCE && cycles < max_cycles) {
            int s2 = vcycle2(lv, 0, L, nu1, nu2);
            if (s2 != REF_OK) { st = s2; break; }
            cycles++;
            ref_residual2(lv[0].n, lv[0].h, P0, lv[0].f, lv[0].r);
            res = ref_norm2_interior(lv[0].n, lv[0].r);
            if (hist) hist[cycles] = res;
            if (!isfinite(res) || res > 10.0 * r0) { st = REF_DIVERGED; break; }
            if (res <= rtol * r0) st = REF_OK;
        }
    }
    if (cycles_out) *cycles_out = cycles;
    if (relres_out) *relres_out = (r0 > 0.0) ? res / r0 : 0.0;
    for (int l = 0; l < L; l++) {
        if (l > 0) free(lv[l].u);
        free(lv[l].f);
        free(lv[l].r);
    }
    free(lv);
    return st;
}

int ref_mg2(const int *n, const double *len, const double *bz0, double *P0, double rtol,
            int max_cycles, int nu1, int nu2, int *cycles_out, double *relres_out, double *hist)
{
    return ref_mg2_edges(n, len, bz0, P0, rtol, max_cycles, nu1, nu2, cycles_out, relres_out, hist, 0);
}

/* One step of the paper's lower-boundary relaxation kernel (Section 4):
 * undamped Jacobi for (11), reading P1 and writing P2.  Interior nodes take
 * the neighbour average weighted by 1/dx^2 and 1/dy^2 plus Bz, divided by
 * 2(1/dx^2 + 1/dy^2); edge nodes are set to zero. */
void ref_jacobi2(const int *n, const double *h, const double *P1, const double *bz, double *P2)
{
    int nx = n[0], ny = n[1];
    double ix2 = 1.0 / (h[0] * h[0]), iy2 = 1.0 / (h[1] * h[1]);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1) {
                AT2(P2, i, j) = 0.0;
                continue;
            }
            AT2(P2, i, j) = ((AT2(P1, i + 1, j) + AT2(P1, i - 1, j)) * ix2 +
                             (AT2(P1, i, j + 1) + AT2(P1, i, j - 1)) * iy2 + AT2(bz, i, j)) /
                            (2.0 * (ix2 + iy2));
        }
}

/* The paper's three steps (Section 2.2): P = 0 everywhere, multigrid for
 * (11) on the base, then multigrid for (8) in the interior.  P is
 * nx*ny*nz; info[0..3] = cycles2d, cycles3d, relres2d, relres3d. */
int ref_solve(const int *n, const double *len, const double *bz0, const double *xi, double alpha,
              double *P, double rtol2, double rtol3, int max_cycles, int nu1, int nu2, double *info)
{
    size_t N = (size_t)n[0] * n[1] * n[2];
    memset(P, 0, sizeof(double) * N);
    int c2 = 0, c3 = 0;
    double r2 = 0.0, r3 = 0.0;
    int st = ref_mg2(n, len, bz0, P, rtol2, max_cycles, nu1, nu2, &c2, &r2, NULL);
    if (st == REF_OK)
        st = ref_mg3(n, len, xi, alpha, P, rtol3, max_cycles, nu1, nu2, &c3, &r3, NULL);
    if (info) {
        info[0] = c2;
        info[1] = c3;
        info[2] = r2;
        info[3] = r3;
    }
    return st;
}

/* ------------------------------------------------------------------ */
/* The general scalar elliptic problem of Section 2.2                   */
/*     a(x) lap u + b(x) u = c(x) in D,   u given on the boundary of D, */
/* with lap the 3D Laplacian (interior) or the 2D one (a face of the    */
/* box: `planar`, one plane of nx*ny nodes, spacings h[0], h[1]).       */
/* ------------------------------------------------------------------ */
/* Reading (the paper states the form, not a discretisation): each
 * interior row is divided by a (a != 0 on interior nodes), giving
 *     lap_h u + beta u = gamma,  beta = b/a,  gamma = c/a,
 * which has the same discrete solution; the multigrid below works on this
 * form (its residual and stopping rule included) with 7-point (5-point)
 * central differences, red-black Gauss-Seidel, the full weighting and
 * interpolation of the problems above, the same coarsening rule, beta
 * sampled at the coarse nodes (as xi is), and an exact solve on the
 * coarsest grid.  The problem must be definite with room to spare: beta
 * at most half the smallest eigenvalue of -lap_h on the coarsest grid
 * (REF_INDEFINITE otherwise), so that every level's operator is definite
 * and no coarse correction over-corrects the lowest mode. */
#define REF_INDEFINITE (-4)

typedef struct {
    int n[3];     /* nodes per axis (n[2] = 1 when planar) */
    double h[3];  /* spacings (h[2] unused when planar) */
    int planar;
} gdom;

static int gen_interior(const gdom *d, int i, int j, int k)
{
    if (i < 1 || i > d->n[0] - 2 || j < 1 || j > d->n[1] - 2) return 0;
    return d->planar ? k == 0 : (k >= 1 && k <= d->n[2] - 2);
}

/* (lap_h u + beta u) at an interior node */
static double gen_op_at(const gdom *d, const double *u, const double *beta, int i, int j, int k)
{
    int nx = d->n[0], ny = d->n[1];
    double c = AT3(u, i, j, k);
    double v = (AT3(u, i + 1, j, k) - 2.0 * c + AT3(u, i - 1, j, k)) / (d->h[0] * d->h[0]) +
               (AT3(u, i, j + 1, k) - 2.0 * c + AT3(u, i, j - 1, k)) / (d->h[1] * d->h[1]);
    if (!d->planar) v += (AT3(u, i, j, k + 1) - 2.0 * c + AT3(u, i, j, k - 1)) / (d->h[2] * d->h[2]);
    return v + AT3(beta, i, j, k) * c;
}

static void gen_dom(gdom *d, const int *n, const double *h, int planar)
{
    d->planar = planar;
    d->n[0] = n[0];
    d->n[1] = n[1];
    d->n[2] = planar ? 1 : n[2];
    d->h[0] = h[0];
    d->h[1] = h[1];
    d->h[2] = planar ? 1.0 : h[2];
}

/* beta = b/a, gamma = c/a on interior nodes, 0 elsewhere; REF_SINGULAR if
 * a vanishes (or any value is not finite) at an interior node. */
int ref_gen_normalise(const int *n, int planar, const double *a, const double *b, const double *c,
                      double *beta, double *gamma)
{
    gdom d;
    double h[3] = {1.0, 1.0, 1.0};
    gen_dom(&d, n, h, planar);
    int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    int st = REF_OK;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double bv = 0.0, gv = 0.0;
                if (gen_interior(&d, i, j, k)) {
                    double av = AT3(a, i, j, k);
                    if (av == 0.0 || !isfinite(av) || !isfinite(AT3(b, i, j, k)) || !isfinite(AT3(c, i, j, k)))
                        st = REF_SINGULAR;
                    bv = AT3(b, i, j, k) / av;
                    gv = AT3(c, i, j, k) / av;
                }
                AT3(beta, i, j, k) = bv;
                AT3(gamma, i, j, k) = gv;
            }
    return st;
}

/* r = gamma - (lap_h u + beta u) on interior nodes, 0 elsewhere */
void ref_gen_residual(const int *n, const double *h, int planar, const double *beta, const double *u,
                      const double *gamma, double *r)
{
    gdom d;
    gen_dom(&d, n, h, planar);
    int nx = d.n[0], ny = d.n[1], nz = d.n[2];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++)
                AT3(r, i, j, k) = gen_interior(&d, i, j, k)
                                      ? AT3(gamma, i, j, k) - gen_op_at(&d, u, beta, i, j, k)
                                      : 0.0;
}

/* nsweeps red-black Gauss-Seidel sweeps in place: every interior node with
 * (i+j+k) even (red) solves its row for itself, then every odd one. */
void ref_gen_rbgs(const int *n, const double *h, int planar, const double *beta, double *u,
                  const double *gamma, int nsweeps)
{
    gdom d;
    gen_dom(&d, n, h, planar);
    int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    double sum = 2.0 / (d.h[0] * d.h[0]) + 2.0 / (d.h[1] * d.h[1]) + (planar ? 0.0 : 2.0 / (d.h[2] * d.h[2]));
    for (int s = 0; s < nsweeps; s++)
        for (int colour = 0; colour < 2; colour++) {
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; k++)
                for (int j = 0; j < ny; j++)
                    for (int i = 0; i < nx; i++) {
                        if (((i + j + k) & 1) != colour || !gen_interior(&d, i, j, k)) continue;
                        /* the node's row: off + (beta - sum) u = gamma, off the
                         * neighbour terms */
                        double off = (AT3(u, i + 1, j, k) + AT3(u, i - 1, j, k)) / (d.h[0] * d.h[0]) +
                                     (AT3(u, i, j + 1, k) + AT3(u, i, j - 1, k)) / (d.h[1] * d.h[1]);
                        if (!planar) off += (AT3(u, i, j, k + 1) + AT3(u, i, j, k - 1)) / (d.h[2] * d.h[2]);
                        AT3(u, i, j, k) = (AT3(gamma, i, j, k) - off) / (AT3(beta, i, j, k) - sum);
                    }
        }
}

/* beta on the next coarser grid: its value at the coincident fine node.
 * kind: STEP_ALL, STEP_XY or STEP_Z (3D); planar grids halve x and y. */
void ref_gen_inject(const int *nf, int planar, int kind, const double *bf, double *bc)
{
    int nx = nf[0], ny = nf[1], nz = planar ? 1 : nf[2];
    int sx = (planar || kind != STEP_Z) ? 2 : 1, sz = (!planar && kind != STEP_XY) ? 2 : 1;
    int ncx = (nx - 1) / sx + 1, ncy = (ny - 1) / sx + 1, ncz = planar ? 1 : (nz - 1) / sz + 1;
    for (int K = 0; K < ncz; K++)
        for (int J = 0; J < ncy; J++)
            for (int I = 0; I < ncx; I++)
                bc[(size_t)I + (size_t)ncx * ((size_t)J + (size_t)ncy * (size_t)K)] = AT3(bf, sx * I, sx * J, sz * K);
}

/* Exact solve of lap_h u + beta u = gamma on the interior nodes of one
 * grid (Gaussian elimination); boundary values of u move to the right. */
int ref_gen_direct(const int *n, const double *h, int planar, const double *beta, double *u,
                   const double *gamma)
{
    gdom d;
    gen_dom(&d, n, h, planar);
    int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    int mx = nx - 2, my = ny - 2, mz = planar ? 1 : nz - 2, k0 = planar ? 0 : 1;
    int m = mx * my * mz;
    double *M = (double *)calloc((size_t)m * m, sizeof(double));
    double *rhs = (double *)calloc((size_t)m, sizeof(double));
    double *x = (double *)calloc((size_t)m, sizeof(double));
    if (!M || !rhs || !x) {
        free(M); free(rhs); free(x);
        return REF_NOMEM;
    }
    double cx = 1.0 / (d.h[0] * d.h[0]), cy = 1.0 / (d.h[1] * d.h[1]), cz = planar ? 0.0 : 1.0 / (d.h[2] * d.h[2]);
    for (int k = k0; k < k0 + mz; k++)
        for (int j = 1; j < ny - 1; j++)
            for (int i = 1; i < nx - 1; i++) {
                int row = (i - 1) + mx * ((j - 1) + my * (k - k0));
                M[(size_t)row * m + row] = AT3(beta, i, j, k) - 2.0 * (cx + cy + cz);
                double rv = AT3(gamma, i, j, k);
                int nb[6][3] = {{i + 1, j, k}, {i - 1, j, k}, {i, j + 1, k}, {i, j - 1, k}, {i, j, k + 1}, {i, j, k - 1}};
                double cf[6] = {cx, cx, cy, cy, cz, cz};
                for (int q = 0; q < (planar ? 4 : 6); q++) {
                    int a = nb[q][0], bb = nb[q][1], c = nb[q][2];
                    if (gen_interior(&d, a, bb, c))
                        M[(size_t)row * m + ((a - 1) + mx * ((bb - 1) + my * (c - k0)))] += cf[q];
                    else
                        rv -= cf[q] * AT3(u, a, bb, c);
                }
                rhs[row] = rv;
            }
    int st = gauss_solve(M, rhs, x, m);
    if (st == REF_OK)
        for (int k = k0; k < k0 + mz; k++)
            for (int j = 1; j < ny - 1; j++)
                for (int i = 1; i < nx - 1; i++) AT3(u, i, j, k) = x[(i - 1) + mx * ((j - 1) + my * (k - k0))];
    free(M); free(rhs); free(x);
    return st;
}

typedef struct {
    int n[3];
    double h[3];
    double *beta, *u, *f, *r;
    size_t N;
    int kind; /* step to the next level (3D); planar steps halve x and y */
} glev;

static void free_glev(glev *lv, int L)
{
    for (int l = 0; l < L; l++) {
        free(lv[l].beta);
        if (l > 0) { free(lv[l].u); free(lv[l].f); }
        free(lv[l].r);
    }
}

/* Levels of the general problem: the coarsening rule of the problems above
 * (every axis halved, or x and y only, or z only, for 3D; x and y for a
 * plane) with beta sampled at the coarse nodes. */
static int build_glev(glev *lv, int L, const int *n, const double *len, int planar, const double *beta0, double *u0,
                      const double *f0)
{
    memset(lv, 0, sizeof(glev) * (size_t)L);
    int kinds[32] = {0};
    if (!planar && ref_levels3(n, len, kinds) != L) return REF_BAD_GRID;
    int nn[3] = {n[0], n[1], planar ? 1 : n[2]};
    for (int l = 0; l < L; l++) {
        for (int a = 0; a < 3; a++) {
            lv[l].n[a] = nn[a];
            lv[l].h[a] = (planar && a == 2) ? 1.0 : len[a] / (double)(nn[a] - 1);
        }
        lv[l].N = (size_t)nn[0] * nn[1] * nn[2];
        lv[l].kind = planar ? STEP_XY : ((l < L - 1) ? kinds[l] : STEP_ALL);
        lv[l].beta = (double *)calloc(lv[l].N, sizeof(double));
        lv[l].r = (double *)calloc(lv[l].N, sizeof(double));
        if (!lv[l].beta || !lv[l].r) return REF_NOMEM;
        if (l == 0) {
            memcpy(lv[0].beta, beta0, sizeof(double) * lv[0].N);
            lv[l].u = u0;
            lv[l].f = (double *)f0;
        } else {
            ref_gen_inject(lv[l - 1].n, planar, lv[l - 1].kind, lv[l - 1].beta, lv[l].beta);
            lv[l].u = (double *)calloc(lv[l].N, sizeof(double));
            lv[l].f = (double *)calloc(lv[l].N, sizeof(double));
            if (!lv[l].u || !lv[l].f) return REF_NOMEM;
        }
        if (planar || lv[l].kind != STEP_Z) {
            nn[0] = (nn[0] - 1) / 2 + 1;
            nn[1] = (nn[1] - 1) / 2 + 1;
        }
        if (!planar && lv[l].kind != STEP_XY) nn[2] = (nn[2] - 1) / 2 + 1;
    }
    return REF_OK;
}

static int gen_vcycle(glev *lv, int l, int L, int planar, int nu1, int nu2)
{
    glev *c = &lv[l];
    if (l == L - 1) return ref_gen_direct(c->n, c->h, planar, c->beta, c->u, c->f);
    ref_gen_rbgs(c->n, c->h, planar, c->beta, c->u, c->f, nu1);
    ref_gen_residual(c->n, c->h, planar, c->beta, c->u, c->f, c->r);
    glev *d = &lv[l + 1];
    if (planar)
        ref_restrict2(c->n, c->r, d->f);
    else if (c->kind == STEP_XY)
        ref_restrict3_xy(c->n, c->r, d->f);
    else if (c->kind == STEP_Z)
        ref_restrict3_z(c->n, c->r, d->f);
    else
        ref_restrict3(c->n, c->r, d->f);
    memset(d->u, 0, sizeof(double) * d->N);
    int st = gen_vcycle(lv, l + 1, L, planar, nu1, nu2);
    if (st != REF_OK) return st;
    if (planar)
        ref_prolong2(d->n, d->u, c->u);
    else if (c->kind == STEP_XY)
        ref_prolong3_xy(d->n, d->u, c->u);
    else if (c->kind == STEP_Z)
        ref_prolong3_z(d->n, d->u, c->u);
    else
        ref_prolong3(d->n, d->u, c->u);
    ref_gen_rbgs(c->n, c->h, planar, c->beta, c->u, c->f, nu2);
    return REF_OK;
}

/* Smallest eigenvalue of -lap_h (zero boundary) on an n-node grid: the
 * sum over axes of (4/h^2) sin^2(pi/(2(n-1))). */
static double gen_lap_lambda_min(const int *n, const double *h, int planar)
{
    const double pi = 3.14159265358979323846;
    double s = 0.0;
    for (int a = 0; a < (planar ? 2 : 3); a++) {
        double t = sin(pi / (2.0 * (double)(n[a] - 1)));
        s += 4.0 / (h[a] * h[a]) * t * t;
    }
    return s;
}

static double ref_norm3_interior_any(const int *n, int planar, const double *r)
{
    return planar ? ref_norm2_interior(n, r) : ref_norm3_interior(n, r);
}

/* Levels of the general problem's hierarchy (3D: the rule above; planar:
 * both axes halved until one has 3 nodes). */
int ref_gen_levels(const int *n, const double *len, int planar)
{
    return planar ? ref_nlevels2(n[0], n[1]) : ref_levels3(n, len, NULL);
}

/* Multigrid solve of a lap u + b u = c for u (x fastest; nz = 1 when planar)
 * in place: u's boundary values are the Dirichlet data, its interior values
 * the initial guess.  len = box lengths (len[2] unused when planar).  Runs
 * V(nu1, nu2) cycles until ||r||/||r0|| <= rtol (r of the divided form) or
 * max_cycles; with rtol < 0 runs exactly max_cycles cycles.  hist (may be
 * NULL) receives ||r_c|| for c = 0..cycles. */
int ref_gen_mg(const int *n, const double *len, int planar, const double *a, const double *b, const double *c,
               double *u, double rtol, int max_cycles, int nu1, int nu2, int *cycles_out, double *relres_out,
               double *hist)
{
    int L = ref_gen_levels(n, len, planar);
    if (L < 1) return REF_BAD_GRID;
    size_t N = (size_t)n[0] * n[1] * (planar ? 1 : n[2]);
    double *beta = (double *)calloc(N, sizeof(double));
    double *gamma = (double *)calloc(N, sizeof(double));
    glev *lv = (glev *)calloc((size_t)L, sizeof(glev));
    if (!beta || !gamma || !lv) {
        free(beta); free(gamma); free(lv);
        return REF_NOMEM;
    }
    int st = ref_gen_normalise(n, planar, a, b, c, beta, gamma);
    if (st == REF_OK) st = build_glev(lv, L, n, len, planar, beta, u, gamma);
    if (st == REF_OK) {
        double bmax = -INFINITY;
        for (size_t e = 0; e < N; e++)
            if (beta[e] > bmax) bmax = beta[e];
        if (!(bmax < 0.5 * gen_lap_lambda_min(lv[L - 1].n, lv[L - 1].h, planar))) st = REF_INDEFINITE;
    }
    int cycles = 0;
    double r0 = 0.0, res = 0.0;
    if (st == REF_OK) {
        glev *f = &lv[0];
        ref_gen_residual(f->n, f->h, planar, f->beta, f->u, f->f, f->r);
        r0 = ref_norm3_interior_any(f->n, planar, f->r);
        res = r0;
        if (hist) hist[0] = r0;
        st = (r0 == 0.0 && rtol >= 0.0) ? REF_OK : REF_NO_CONVERGENCE;
        while (st == REF_NO_CONVERGENCE && cycles < max_cycles) {
            int s2 = gen_vcycle(lv, 0, L, planar, nu1, nu2);
            if (s2 != REF_OK) { st = s2; break; }
            cycles++;
            ref_gen_residual(f->n, f->h, planar, f->beta, f->u, f->f, f->r);
            res = ref_norm3_interior_any(f->n, planar, f->r);
            if (hist) hist[cycles] = res;
            if (!isfinite(res) || res > 10.0 * r0) { st = REF_DIVERGED; break; }
            if (rtol >= 0.0 && res <= rtol * r0) st = REF_OK;
        }
        if (rtol < 0.0 && st == REF_NO_CONVERGENCE) st = REF_OK;
    }
    if (cycles_out) *cycles_out = cycles;
    if (relres_out) *relres_out = (r0 > 0.0) ? res / r0 : 0.0;
    free_glev(lv, L);
    free(lv);
    free(beta);
    free(gamma);
    return st;
}
