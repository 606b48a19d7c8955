// C-ABI of libmhs: plans, validation, coefficient tables, the coarsest-grid
// inverse, V-cycle programs and the solve drivers.
//
// The procedure follows Section 2.2: P = 0 everywhere (step 1), multigrid on
// the lower-boundary equation (11) (step 2), multigrid on the interior
// equation (8) with the base plane as Dirichlet data (step 3), then the field
// recovery of equations (5), (6), (9), (10).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "plan.h"

using namespace mhs;

namespace mhs {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

constexpr size_t kStagingBytes = 1 << 20;
// Workgroups a stencil launch aims for: about as many as fit on the chip at
// once (4-5 per CU on 256 CUs), so that one round of resident groups covers
// the grid with long z-marches (fewer re-read halo planes, no tail round).
// The field recovery, whose groups hold more LDS, prefers two rounds.
#ifndef MHS_TARGET_GROUPS
#define MHS_TARGET_GROUPS 1024
#endif
constexpr int kTargetGroups = MHS_TARGET_GROUPS;
#ifndef MHS_COARSE_TARGET_GROUPS
#define MHS_COARSE_TARGET_GROUPS 1024
#endif
constexpr int kCoarseTargetGroups = MHS_COARSE_TARGET_GROUPS;
// The same per request for levels >= 1 in merged launches of the batch
// (many requests per launch fill the chip with fewer groups each).
#ifndef MHS_BATCH_COARSE_TARGET_GROUPS
#define MHS_BATCH_COARSE_TARGET_GROUPS 128
#endif
constexpr int kBatchCoarseTargetGroups = MHS_BATCH_COARSE_TARGET_GROUPS;
constexpr int kFieldsTargetGroups = 2048;
// Largest coarsest grid (unknowns) a model may cut the 3D hierarchy to.
constexpr int kMaxCutCoarse = 512;

// LDS bytes of a bottom solver starting at level l: u and f of every level
// from l down with their coefficient tables (4 nz each), plus a residual
// array of level l.
size_t bottom_lds(const Hierarchy &h, int l)
{
    size_t n = 0;
    for (int q = l; q < h.L; ++q) n += 2 * h.lv[q].N + 4 * (size_t)h.lv[q].n[2];
    return 8 * (n + h.lv[l].N);
}

int chunk(int planes, int xy_tiles, int cap, int target = kTargetGroups)
{
    const long want = ((long)planes * xy_tiles + target - 1) / target;
    return (int)std::max(1L, std::min((long)cap, want));
}

bool valid_axis(int n)
{
    if (n < 5) return false;
    const int m = n - 1;
    return (m & (m - 1)) == 0;
}

int check_grid(const mhs_grid *g)
{
    if (!g) return fail(MHS_ERR_INVALID_ARG, "grid is NULL");
    if (!valid_axis(g->nx) || !valid_axis(g->ny) || !valid_axis(g->nz))
        return fail(MHS_ERR_GRID, "every axis needs 2^L+1 nodes with L >= 2 (got %d x %d x %d)", g->nx, g->ny,
                    g->nz);
    if (!(g->lx > 0 && g->ly > 0 && g->lz > 0) || !std::isfinite(g->lx) || !std::isfinite(g->ly) ||
        !std::isfinite(g->lz))
        return fail(MHS_ERR_INVALID_ARG, "box lengths must be positive and finite");
    const double npts = (double)g->nx * g->ny * g->nz;
    // at most 2e9 nodes (32-bit node indices); with nz >= 5 an FP64 x-y
    // plane then stays under 4 GB (the kernels' 32-bit byte offsets)
    if (npts > 2.0e9) return fail(MHS_ERR_GRID, "grid too large (%g nodes)", npts);
    return MHS_OK;
}

// Geometry of a hierarchy (no buffers).  A 2D step halves both axes.  A 3D
// step halves every axis, except that it keeps z when dz^2 >= 2 max(dx, dy)^2
// (x-y semicoarsening) and keeps x and y when 2 dz^2 <= min(dx, dy)^2 (z
// semicoarsening): the paper does not say how coarse grids are built, and
// halving only the finer axes brings a grid with dz != dx toward equal
// spacing, where point red-black smoothing reduces the oscillatory error in
// every direction.  Coarsening stops when an axis to be halved has 3 nodes.
int build_geometry(Hierarchy &h, const int n0[3], const double len[3], bool planar)
{
    h = Hierarchy();
    h.planar = planar;
    int n[3] = {n0[0], n0[1], planar ? 1 : n0[2]};
    int L = 0, zs = 0;
    for (;;) {
        if (L >= kMaxLevels) return fail(MHS_ERR_GRID, "too many levels");
        Level &lv = h.lv[L];
        for (int a = 0; a < 3; ++a) lv.n[a] = n[a];
        lv.h[0] = len[0] / (n[0] - 1);
        lv.h[1] = len[1] / (n[1] - 1);
        lv.h[2] = planar ? 1.0 : len[2] / (n[2] - 1);
        lv.N = (size_t)n[0] * n[1] * n[2];
        lv.zs = zs;
        ++L;
        const double hmax = std::max(lv.h[0], lv.h[1]), hmin = std::min(lv.h[0], lv.h[1]);
        const double hz2 = lv.h[2] * lv.h[2];
        const bool keepz = !planar && hz2 >= 2.0 * hmax * hmax;
        const bool keepxy = !planar && !keepz && 2.0 * hz2 <= hmin * hmin;
        const bool more = (keepxy || (n[0] > 3 && n[1] > 3)) && (planar || keepz || n[2] > 3);
        if (!more) break;
        lv.keepz = keepz;
        lv.keepxy = keepxy;
        if (!keepxy) {
            n[0] = (n[0] - 1) / 2 + 1;
            n[1] = (n[1] - 1) / 2 + 1;
        }
        if (!planar && !keepz) {
            n[2] = (n[2] - 1) / 2 + 1;
            ++zs;
        }
    }
    h.L = L;
    if (L < 2) return fail(MHS_ERR_GRID, "grid too small for multigrid");
    const Level &c = h.lv[L - 1];
    h.m = (c.n[0] - 2) * (c.n[1] - 2) * (planar ? 1 : c.n[2] - 2);
    if (h.m > kMaxCoarse)
        return fail(MHS_ERR_GRID, "coarsest grid has %d unknowns (max %d): axes too unequal", h.m, kMaxCoarse);
    h.b = -1;
    for (int l = 1; l < L; ++l)
        if (bottom_lds(h, l) <= (size_t)kBottomLdsMax) {
            h.b = l;
            break;
        }
    if (h.b < 0) return fail(MHS_ERR_GRID, "coarsest grid too large for the LDS bottom solver");
    h.lds_bytes = (int)bottom_lds(h, h.b);
    h.Lgeo = h.L;
    h.bgeo = h.b;
    h.mcap = h.m;
    for (int l = 1; l < L; ++l) {
        const Level &q = h.lv[l];
        const int mq = (q.n[0] - 2) * (q.n[1] - 2) * (planar ? 1 : q.n[2] - 2);
        if (mq <= kMaxCutCoarse) h.mcap = std::max(h.mcap, mq);
    }
    for (int l = 0; l < L; ++l) {
        Level &lv = h.lv[l];
        if (planar) {
            lv.st[0] = ceil_div(lv.n[0] - 2, kTX);
            lv.st[1] = ceil_div(lv.n[1] - 2, kTY2);
            lv.ity = lv.st[1];
            lv.st[2] = 1;
            lv.kz = 1;
            lv.stz_b = 1;
            lv.kz_b = 1;
        } else {
            lv.st[0] = ceil_div(lv.n[0] - 2, kTX);
            lv.st[1] = ceil_div(lv.n[1] - 2, kSTY);
            lv.ity = ceil_div(lv.n[1] - 2, kTY);
            // z-chunks sized in kTX x kTY tiles of kThreads threads: the
            // smoother's taller tiles give fewer, larger workgroups over the
            // same number of threads
            lv.kz = chunk(lv.n[2] - 2, lv.st[0] * lv.ity, kKZ, l == 0 ? kTargetGroups : kCoarseTargetGroups);
            lv.st[2] = ceil_div(lv.n[2] - 2, lv.kz);
            lv.kz_b = l == 0 ? lv.kz : chunk(lv.n[2] - 2, lv.st[0] * lv.ity, kKZ, kBatchCoarseTargetGroups);
            lv.stz_b = ceil_div(lv.n[2] - 2, lv.kz_b);
        }
        if (l + 1 < L) {
            const Level &c2 = h.lv[l + 1];
            lv.rt[0] = ceil_div(c2.n[0] - 2, kCX);
            lv.rt[1] = ceil_div(c2.n[1] - 2, kCY);
            if (planar) {
                lv.rt[2] = 1;
                lv.kc = 1;
                lv.rtz_b = 1;
                lv.kc_b = 1;
            } else {
                lv.kc = chunk(c2.n[2] - 2, lv.rt[0] * lv.rt[1], kKC, l == 0 ? kTargetGroups : kCoarseTargetGroups);
                lv.rt[2] = ceil_div(c2.n[2] - 2, lv.kc);
                lv.kc_b = l == 0 ? lv.kc : chunk(c2.n[2] - 2, lv.rt[0] * lv.rt[1], kKC, kBatchCoarseTargetGroups);
                lv.rtz_b = ceil_div(c2.n[2] - 2, lv.kc_b);
            }
        }
    }
    return MHS_OK;
}

// Lay out the buffers of a hierarchy.  paths: bit 0 = FP64 cycles, bit 1 =
// FP32 inner cycles.  Level 0's iterate is the caller's array (set per call);
// its twin is allocated whenever any path exists.
void carve_hierarchy(Hierarchy &h, Carver &cv, int paths)
{
    const int L = h.L, b = h.b;
    Level &l0 = h.lv[0];
    l0.t[kF64] = cv.take<double>(l0.N);
    if (h.planar) l0.f[kF64] = cv.take<double>(l0.N);
    for (int p = 0; p < 2; ++p) {
        if (!(paths & (1 << p))) continue;
        const size_t es = p == kF64 ? sizeof(double) : sizeof(float);
        if (p == kF32) {
            l0.u[kF32] = cv.take<char>(l0.N * es);
            l0.t[kF32] = cv.take<char>(l0.N * es);
            l0.f[kF32] = cv.take<char>(l0.N * es);
        }
        for (int l = 1; l <= b; ++l) {
            Level &lv = h.lv[l];
            lv.u[p] = cv.take<char>(lv.N * es);
            lv.f[p] = cv.take<char>(lv.N * es);
            if (l < b) lv.t[p] = cv.take<char>(lv.N * es);
        }
    }
    // the model's tables, then the coarsest inverse, in one contiguous range
    // from level 0's FP64 table: a model is uploaded with a single copy
    for (int l = 0; l < L; ++l) {
        Level &lv = h.lv[l];
        lv.coef64 = cv.take<double>(4 * (size_t)lv.n[2]);
        if (paths & 2) lv.coef32 = cv.take<float>(4 * (size_t)lv.n[2]);
    }
    h.minv = cv.take<double>((size_t)h.mcap * h.mcap);
    h.npart = std::max(l0.sweep_tiles(), l0.ir_tiles());
    h.partials = cv.take<double>(h.npart);
}

size_t carve_plan(mhs_plan *p, char *base, int precisions)
{
    Carver cv{base};
    int paths = 0;
    if (precisions & MHS_PREC_FP64) paths |= 1;
    if (precisions & MHS_PREC_MIXED) paths |= 2;
    carve_hierarchy(p->h3, cv, paths);
    carve_hierarchy(p->h2, cv, 1);
    p->d_fields_tab = cv.take<double>(4 * (size_t)p->grid.nz);
    p->scratch_npart = std::max(p->h3.npart, p->h2.npart);
    p->d_scratch_norm = cv.take<double>(p->scratch_npart);
    p->stage.dev = cv.take<char>(kStagingBytes);
    p->stage.cap = kStagingBytes;
    if (precisions & MHS_PLAN_GENERAL) gen_create(p, cv);
    return cv.off + kAlign;
}

int geometry(mhs_plan *p, const mhs_grid *g)
{
    p->grid = *g;
    const int n0[3] = {g->nx, g->ny, g->nz};
    const double len[3] = {g->lx, g->ly, g->lz};
    int st = build_geometry(p->h3, n0, len, false);
    if (st) return st;
    return build_geometry(p->h2, n0, len, true);
}

// ---- coefficient tables and the coarsest-grid inverse --------------------------

// cx_k = (1 - xi_k)/dx^2, cy_k = (1 - xi_k)/dy^2, d_k = alpha^2 - 2cx - 2cy - 2cz
// (equation (8) at level l, xi sampled at the level's nodes: xi_l[k] = xi[k 2^zs],
// zs the number of steps above l that halved z).
void level_coef(const Hierarchy &h, int l, double alpha, const double *xi, std::vector<double> &out,
                double &cz)
{
    const Level &lv = h.lv[l];
    const int nz = lv.n[2];
    out.assign(4 * (size_t)nz, 0.0);
    const double ix2 = 1.0 / (lv.h[0] * lv.h[0]), iy2 = 1.0 / (lv.h[1] * lv.h[1]);
    cz = h.planar ? 0.0 : 1.0 / (lv.h[2] * lv.h[2]);
    for (int k = 0; k < nz; ++k) {
        const double x = h.planar ? 0.0 : xi[(size_t)k << lv.zs];
        const double cx = (1.0 - x) * ix2, cy = (1.0 - x) * iy2;
        const double a2 = h.planar ? 0.0 : alpha * alpha;
        const double d = a2 - 2.0 * cx - 2.0 * cy - 2.0 * cz;
        out[4 * k] = cx;
        out[4 * k + 1] = cy;
        out[4 * k + 2] = d;
        out[4 * k + 3] = 1.0 / d;
    }
}

// Inverse of the coarsest operator A (m x m, interior nodes x fastest) by
// Cholesky of -A (which is symmetric positive definite when (8) is definite
// on that grid) followed by triangular solves against the identity.
int coarse_inverse(const Hierarchy &h, const std::vector<double> &coef, double cz, std::vector<double> &minv)
{
    const Level &c = h.lv[h.L - 1];
    const int mx = c.n[0] - 2, my = c.n[1] - 2, mz = h.planar ? 1 : c.n[2] - 2;
    const int m = mx * my * mz;
    std::vector<double> M((size_t)m * m, 0.0); // -A
    for (int kk = 0; kk < mz; ++kk)
        for (int jj = 0; jj < my; ++jj)
            for (int ii = 0; ii < mx; ++ii) {
                const int r = ii + mx * (jj + my * kk);
                const int k = h.planar ? 0 : kk + 1;
                const double cx = coef[4 * k], cy = coef[4 * k + 1], d = coef[4 * k + 2];
                M[(size_t)r * m + r] = -d;
                if (ii > 0) M[(size_t)r * m + r - 1] = -cx;
                if (ii + 1 < mx) M[(size_t)r * m + r + 1] = -cx;
                if (jj > 0) M[(size_t)r * m + r - mx] = -cy;
                if (jj + 1 < my) M[(size_t)r * m + r + mx] = -cy;
                if (kk > 0) M[(size_t)r * m + r - mx * my] = -cz;
                if (kk + 1 < mz) M[(size_t)r * m + r + mx * my] = -cz;
            }
    // Cholesky M = G G^T (lower G stored in M)
    for (int j = 0; j < m; ++j) {
        double s = M[(size_t)j * m + j];
        for (int q = 0; q < j; ++q) s -= M[(size_t)j * m + q] * M[(size_t)j * m + q];
        if (!(s > 0.0))
            return fail(MHS_ERR_INDEFINITE, "coarsest operator is not definite: alpha^2 too large for this box");
        const double g = std::sqrt(s);
        M[(size_t)j * m + j] = g;
        for (int i = j + 1; i < m; ++i) {
            double t = M[(size_t)i * m + j];
            for (int q = 0; q < j; ++q) t -= M[(size_t)i * m + q] * M[(size_t)j * m + q];
            M[(size_t)i * m + j] = t / g;
        }
    }
    minv.assign((size_t)m * m, 0.0);
    std::vector<double> y(m);
    for (int col = 0; col < m; ++col) {
        for (int i = 0; i < m; ++i) {
            double s = (i == col) ? 1.0 : 0.0;
            for (int q = 0; q < i; ++q) s -= M[(size_t)i * m + q] * y[q];
            y[i] = s / M[(size_t)i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double s = y[i];
            for (int q = i + 1; q < m; ++q) s -= M[(size_t)q * m + i] * y[q];
            y[i] = s / M[(size_t)i * m + i];
        }
        // A^{-1} = -(-A)^{-1}
        for (int i = 0; i < m; ++i) minv[(size_t)i * m + col] = -y[i];
    }
    return MHS_OK;
}

// Smallest eigenvalue of -[(1 - xi(z)) (d2x + d2y) + d2z] on the interior
// unknowns of level l (the operator of (8) without the alpha^2 term).  The
// operator separates: an in-plane sine mode of eigenvalue lam turns it into
// the symmetric tridiagonal T = -d2z + lam diag(1 - xi_k), whose eigenvalues
// grow with lam (1 - xi > 0), so the minimum sits at the smallest in-plane
// eigenvalue.  T = iz2 K + D with K = tridiag(-1, 2, -1) and D diagonal, so
// Weyl's inequality puts its smallest eigenvalue at or above
// iz2 mu1 + min D (mu1 = 4 sin^2(pi / (2 (m + 1))), the smallest of K), and
// the Rayleigh quotient of K's first eigenvector at or below
// iz2 mu1 + (its weighted mean of D): a bracket that is exact for constant
// xi.  Passes of Sturm counts (the number of negative pivots of T - x I) at
// three points narrow it by four; callers narrow it only as far as their
// decisions need.
struct LambdaBracket {
    std::vector<double> a;
    double b2 = 0.0, lo = 0.0, hi = 0.0;
    int m = 0;
    LambdaBracket(const Hierarchy &h, int l, const double *xi, const double len[3])
    {
        const Level &lv = h.lv[l];
        auto lam1 = [](double hh, double length) {
            const double s = std::sin(3.14159265358979323846 * hh / (2.0 * length));
            return 4.0 / (hh * hh) * s * s;
        };
        const double lxy = lam1(lv.h[0], len[0]) + lam1(lv.h[1], len[1]);
        m = lv.n[2] - 2;
        const double iz2 = 1.0 / (lv.h[2] * lv.h[2]);
        const double sk = std::sin(3.14159265358979323846 / (2.0 * (m + 1)));
        const double base = iz2 * 4.0 * sk * sk;
        a.resize((size_t)m);
        double dmin = 0.0, amin = 0.0, wsum = 0.0, wd = 0.0;
        for (int q = 0; q < m; ++q) {
            const double d = (1.0 - xi[(size_t)(q + 1) << lv.zs]) * lxy;
            a[(size_t)q] = 2.0 * iz2 + d;
            dmin = q == 0 ? d : std::min(dmin, d);
            amin = q == 0 ? a[0] : std::min(amin, a[(size_t)q]); // Rayleigh quotient of a unit vector
            const double v = std::sin(3.14159265358979323846 * (q + 1) / (m + 1));
            wsum += v * v;
            wd += v * v * d;
        }
        b2 = iz2 * iz2;
        // a relative margin of 1e-12 keeps the rounded bounds outside
        lo = std::max(0.0, (base + dmin) * (1.0 - 1e-12));
        hi = std::min(amin, (base + wd / wsum) * (1.0 + 1e-12));
        if (!(hi > lo)) hi = lo * (1.0 + 1e-12) + 1e-300;
    }
    bool fine() const { return !(hi - lo > 1e-14 * hi); }
    // one pass: three pivot recurrences (their divisions overlap) decide in
    // which quarter of [lo, hi] the smallest eigenvalue lies
    void pass()
    {
        const double w = hi - lo;
        const double x[3] = {lo + 0.25 * w, lo + 0.5 * w, lo + 0.75 * w};
        double d[3] = {1.0, 1.0, 1.0};
        int cnt[3] = {0, 0, 0};
        for (int q = 0; q < m; ++q) {
            for (int c = 0; c < 3; ++c) {
                double v = (a[(size_t)q] - x[c]) - (q ? b2 / d[c] : 0.0);
                if (v == 0.0) v = -1e-300;
                cnt[c] += v < 0.0;
                d[c] = v;
            }
        }
        if (cnt[0] >= 1) {
            hi = x[0];
        } else if (cnt[1] >= 1) {
            lo = x[0];
            hi = x[1];
        } else if (cnt[2] >= 1) {
            lo = x[1];
            hi = x[2];
        } else {
            lo = x[2];
        }
    }
    // narrowed to 1e-14 of hi: lo is then the smallest eigenvalue
    double value()
    {
        for (int it = 0; it < 100 && !fine(); ++it) pass();
        return lo;
    }
};

double level_lambda_min(const Hierarchy &h, int l, const double *xi, const double len[3])
{
    LambdaBracket b(h, l, xi, len);
    return b.value();
}

// Use levels 0..L-1 of a hierarchy: the bottom solver starts at the first
// level whose bottom part fits the LDS, and the coarsest grid is L-1.
int set_depth(Hierarchy &h, int L)
{
    if (L < 2 || L > h.Lgeo) return fail(MHS_ERR_INDEFINITE, "no usable multigrid hierarchy");
    Hierarchy t = h; // decide on a copy; commit only a consistent depth
    t.L = L;
    const Level &c = t.lv[L - 1];
    t.m = (c.n[0] - 2) * (c.n[1] - 2) * (t.planar ? 1 : c.n[2] - 2);
    if (t.m > t.mcap)
        return fail(MHS_ERR_INDEFINITE,
                    "alpha^2 is too close to resonance: the coarsest grid that still represents the lowest mode "
                    "has %d unknowns (max %d)", t.m, t.mcap);
    t.b = -1;
    for (int l = 1; l < L; ++l)
        if (bottom_lds(t, l) <= (size_t)kBottomLdsMax) {
            t.b = l;
            break;
        }
    if (t.b < 0 || t.b > t.bgeo) return fail(MHS_ERR_INDEFINITE, "coarsest usable grid too large for the bottom solver");
    h.L = t.L;
    h.m = t.m;
    h.b = t.b;
    h.lds_bytes = (int)bottom_lds(t, t.b);
    return MHS_OK;
}

// Depth of the 3D hierarchy for a model (a reading: the paper is silent on
// the coarse grids).  The operator of (8) must be definite on the grid:
// alpha^2 below the smallest eigenvalue lambda_0 of
// -[(1 - xi)(d2x + d2y) + d2z].  Coarse grids under-resolve the lowest mode,
// so their smallest eigenvalue lambda_l drops as the grid coarsens; a coarse
// correction built on a level with lambda_l - alpha^2 below half of
// lambda_0 - alpha^2 over-corrects that mode more than twofold and the
// cycle stops contracting (near resonance).  The hierarchy therefore stops
// above the first such level, whose parent is solved exactly.
constexpr double kResonanceRatio = 0.5;

int model_depth(const Hierarchy &h, const mhs_grid &g, const mhs_model *model, int *depth, double *lambda0)
{
    const double len[3] = {g.lx, g.ly, g.lz};
    const double a2 = model->alpha * model->alpha;
    // each comparison narrows the brackets until it is decided by them, or
    // both are at 1e-14 width and their lower ends decide it
    LambdaBracket b0(h, 0, model->xi, len);
    if (lambda0) *lambda0 = b0.value();
    while (!(b0.lo > a2) && !(b0.hi <= a2) && !b0.fine()) b0.pass();
    if (!(a2 < b0.lo))
        return fail(MHS_ERR_INDEFINITE, "alpha^2 = %g is not below the smallest eigenvalue %g of (8) on the grid", a2,
                    b0.value());
    int L = h.Lgeo;
    for (int l = 1; l < h.Lgeo; ++l) {
        LambdaBracket bl(h, l, model->xi, len);
        bool stop;
        for (;;) {
            if (bl.lo - a2 >= kResonanceRatio * (b0.hi - a2)) {
                stop = false;
                break;
            }
            if (bl.hi - a2 < kResonanceRatio * (b0.lo - a2)) {
                stop = true;
                break;
            }
            if (bl.fine() && b0.fine()) {
                stop = !(bl.lo - a2 >= kResonanceRatio * (b0.lo - a2));
                break;
            }
            if (!bl.fine() && (b0.fine() || (bl.hi - bl.lo) / bl.hi >= (b0.hi - b0.lo) / b0.hi))
                bl.pass();
            else
                b0.pass();
        }
        if (stop) {
            L = l;
            break;
        }
    }
    if (L < 2) return fail(MHS_ERR_INDEFINITE, "alpha^2 = %g is too close to resonance for any coarse grid", a2);
    *depth = L;
    return MHS_OK;
}

int prepare_model(mhs_plan *p, const mhs_model *model, ModelUpload &up)
{
    up.parts.clear();
    up.data.clear();
    const int nz = p->grid.nz;
    Hierarchy &h = p->h3;
    const bool same = p->cache.valid && p->cache.alpha == model->alpha &&
                      std::equal(p->cache.xi.begin(), p->cache.xi.end(), model->xi);
    if (same) return MHS_OK;
    int depth = 0;
    int st0 = model_depth(h, p->grid, model, &depth, nullptr);
    if (st0) return st0;
    if ((st0 = set_depth(h, depth))) return st0;
    // the tables lie in one device range from level 0's FP64 table (the
    // plan's layout); the host image mirrors it, padding zeroed, so that a
    // single copy uploads the model
    char *const base = (char *)h.lv[0].coef64;
    bool contiguous = true;
    auto add = [&](void *dst, const void *src, size_t bytes) {
        if ((char *)dst < base) {
            contiguous = false;
            return;
        }
        const size_t off = (size_t)((char *)dst - base);
        if (up.data.size() < off + bytes) up.data.resize(off + bytes);
        std::memcpy(up.data.data() + off, src, bytes);
    };
    std::vector<double> tab, minv;
    std::vector<float> t32;
    for (int l = 0; l < h.L; ++l) {
        double cz = 0.0;
        level_coef(h, l, model->alpha, model->xi, tab, cz);
        h.lv[l].cz = cz;
        add(h.lv[l].coef64, tab.data(), tab.size() * sizeof(double));
        if (h.lv[l].coef32) {
            t32.assign(tab.begin(), tab.end());
            add(h.lv[l].coef32, t32.data(), t32.size() * sizeof(float));
        }
        if (l == h.L - 1) {
            int st = coarse_inverse(h, tab, cz, minv);
            if (st) return st;
            add(h.minv, minv.data(), minv.size() * sizeof(double));
        }
    }
    if (!contiguous) return fail(MHS_ERR_WORKSPACE, "model tables are not laid out from level 0's table");
    up.parts.push_back({base, 0, up.data.size()});
    // the plan's tables will hold this model once the copies have run
    p->cache.valid = true;
    p->cache.alpha = model->alpha;
    p->cache.xi.assign(model->xi, model->xi + nz);
    return MHS_OK;
}

void invalidate_model(mhs_plan *p) { p->cache.valid = false; }

int upload_model(mhs_plan *p, const mhs_model *model, hipStream_t s)
{
    ModelUpload up;
    int st = prepare_model(p, model, up);
    if (st) return st;
    for (const ModelUpload::Part &q : up.parts)
        HIPCHK(hipMemcpyAsync(q.dst, up.data.data() + q.off, q.bytes, hipMemcpyHostToDevice, s));
    // pageable sources: make sure the copies have consumed them before return
    if (!up.parts.empty()) HIPCHK(hipStreamSynchronize(s));
    return MHS_OK;
}

int upload_planar(mhs_plan *p, hipStream_t s)
{
    Hierarchy &h = p->h2;
    std::vector<double> tab, minv;
    for (int l = 0; l < h.L; ++l) {
        double cz = 0.0;
        level_coef(h, l, 0.0, nullptr, tab, cz);
        h.lv[l].cz = 0.0;
        HIPCHK(hipMemcpyAsync(h.lv[l].coef64, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
        if (l == h.L - 1) {
            int st = coarse_inverse(h, tab, 0.0, minv);
            if (st) return st;
            HIPCHK(hipMemcpyAsync(h.minv, minv.data(), minv.size() * sizeof(double), hipMemcpyHostToDevice, s));
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    return MHS_OK;
}

int validate_model(const mhs_plan *p, const mhs_model *m, bool need_fields)
{
    if (!m || !m->xi) return fail(MHS_ERR_INVALID_ARG, "model or model->xi is NULL");
    if (!std::isfinite(m->alpha)) return fail(MHS_ERR_INVALID_ARG, "alpha is not finite");
    const int nz = p->grid.nz;
    for (int k = 0; k < nz; ++k)
        if (!std::isfinite(m->xi[k])) return fail(MHS_ERR_INVALID_ARG, "xi[%d] is not finite", k);
    for (int k = 1; k < nz - 1; ++k)
        if (!(m->xi[k] < 1.0))
            return fail(MHS_ERR_NOT_ELLIPTIC, "xi(z_%d) = %g >= 1: equation (8) is not elliptic", k, m->xi[k]);
    if (need_fields) {
        if (!m->dxi || !m->pb || !m->rhob) return fail(MHS_ERR_INVALID_ARG, "dxi, pb and rhob are required");
        if (!(m->mu0 > 0.0) || !(m->g > 0.0)) return fail(MHS_ERR_INVALID_ARG, "mu0 and g must be positive");
        for (int k = 0; k < nz; ++k)
            if (!std::isfinite(m->dxi[k]) || !std::isfinite(m->pb[k]) || !std::isfinite(m->rhob[k]))
                return fail(MHS_ERR_INVALID_ARG, "non-finite model table entry at k = %d", k);
    }
    return MHS_OK;
}

int validate_opts(const mhs_opts *o)
{
    if (!o) return fail(MHS_ERR_INVALID_ARG, "opts is NULL");
    if (o->precision != MHS_PREC_FP64 && o->precision != MHS_PREC_MIXED)
        return fail(MHS_ERR_INVALID_ARG, "precision must be MHS_PREC_FP64 or MHS_PREC_MIXED");
    if (o->nu1 < 1 || o->nu2 < 1 || o->nu1 > 16 || o->nu2 > 16)
        return fail(MHS_ERR_INVALID_ARG, "nu1 and nu2 must be in 1..16");
    if (o->max_cycles < 0) return fail(MHS_ERR_INVALID_ARG, "max_cycles must be >= 0");
    if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol)) return fail(MHS_ERR_INVALID_ARG, "rtol must be >= 0");
    if (o->inner_cycles < 1 || o->inner_cycles > 16) return fail(MHS_ERR_INVALID_ARG, "inner_cycles must be in 1..16");
    if (o->check_every < 0) return fail(MHS_ERR_INVALID_ARG, "check_every must be >= 0");
    if (o->faces != MHS_FACES_ZERO && o->faces != MHS_FACES_GIVEN)
        return fail(MHS_ERR_INVALID_ARG, "faces must be MHS_FACES_ZERO or MHS_FACES_GIVEN");
    if (o->graph != 0 && o->graph != 1) return fail(MHS_ERR_INVALID_ARG, "graph must be 0 or 1");
    return MHS_OK;
}

// ---- programs -----------------------------------------------------------------

LevelItem level_item(const Hierarchy &h, int l, int path)
{
    const Level &lv = h.lv[l];
    LevelItem it{};
    it.coef = path == kF64 ? (const void *)lv.coef64 : (const void *)lv.coef32;
    it.cz = lv.cz;
    it.nx = lv.n[0];
    it.ny = lv.n[1];
    it.nz = lv.n[2];
    if (l + 1 < h.L) {
        it.ncx = h.lv[l + 1].n[0];
        it.ncy = h.lv[l + 1].n[1];
        it.ncz = h.lv[l + 1].n[2];
    }
    return it;
}

void add_sweep(Program &pg, Staging &st, const Hierarchy &h, int l, int path, const void *uin, void *uout,
               const void *f, const void *ec, int flags, SolveState *state, double *partials)
{
    LevelItem it = level_item(h, l, path);
    const Level &lv = h.lv[l];
    it.u_in = uin;
    it.u_out = uout;
    it.f = f;
    it.ec = ec;
    it.state = state;
    it.partials = partials;
    // levels >= 1 have no reductions: their z-chunking does not change a
    // result, so merged launches may use the batched chunking
    const bool bt = h.batched && l > 0;
    it.ntx = lv.st[0];
    it.nty = lv.st[1];
    it.ntz = bt ? lv.stz_b : lv.st[2];
    it.kz = bt ? lv.kz_b : lv.kz;
    it.tile_base = 0;
    const LevelItem *d = st.put(it);
    if (!d) {
        pg.ok = false;
        return;
    }
    Launch L{};
    L.kind = h.planar ? Launch::kSweep2 : Launch::kSweep3;
    L.flags = flags | (f ? kHasF : 0);
    L.dbl = path == kF64;
    L.items = d;
    L.nitems = 1;
    L.ntiles = it.ntx * it.nty * it.ntz;
    L.prof = (l == 0 && !h.planar) ? MHS_PROF_SMOOTH_L0 : MHS_PROF_COARSE;
    {
        const double es = path == kF64 ? 8.0 : 4.0;
        double words = 1.0;                      // write u
        if (!(L.flags & kZeroIn)) words += 1.0;  // read u
        if (L.flags & kHasF) words += 1.0;       // read f
        L.bytes = es * words * (double)lv.N;
        if ((L.flags & kProlong) && l + 1 < h.L) L.bytes += es * (double)h.lv[l + 1].N;
    }
    L.pre = (flags & kNorm) != 0;
    pg.launches.push_back(L);
}

void add_restrict(Program &pg, Staging &st, const Hierarchy &h, int l, int path, const void *u, const void *f,
                  void *fc, SolveState *state)
{
    LevelItem it = level_item(h, l, path);
    const Level &lv = h.lv[l];
    it.u_in = u;
    it.f = f;
    it.u_out = fc;
    it.state = state;
    const bool bt = h.batched && l > 0;
    const bool zonly = !h.planar && lv.keepxy;
    if (zonly) { // one thread per coarse interior node
        const Level &c = h.lv[l + 1];
        it.ntx = ceil_div((c.n[0] - 2) * (c.n[1] - 2) * (c.n[2] - 2), kThreads);
        it.nty = it.ntz = it.kz = 1;
    } else {
        it.ntx = lv.rt[0];
        it.nty = lv.rt[1];
        it.ntz = bt ? lv.rtz_b : lv.rt[2];
        it.kz = bt ? lv.kc_b : lv.kc;
    }
    const LevelItem *d = st.put(it);
    if (!d) {
        pg.ok = false;
        return;
    }
    Launch L{};
    L.kind = h.planar ? Launch::kRestrict2 : zonly ? Launch::kRestrict3Z : Launch::kRestrict3;
    L.flags = (f ? kRestrictHasF : 0) | (lv.keepz ? kRestrictKeepZ : 0);
    L.dbl = path == kF64;
    L.items = d;
    L.ntiles = it.ntx * it.nty * it.ntz;
    L.prof = (l == 0 && !h.planar) ? MHS_PROF_RESTRICT_L0 : MHS_PROF_COARSE;
    {
        const double es = path == kF64 ? 8.0 : 4.0;
        L.bytes = es * ((f ? 2.0 : 1.0) * (double)lv.N + (double)h.lv[l + 1].N);
    }
    pg.launches.push_back(L);
}

BottomItem bottom_item(const Hierarchy &h, int path, const void *f_top, void *u_top, int nu1, int nu2,
                       SolveState *state)
{
    BottomItem b{};
    b.f_top = f_top;
    b.u_top = u_top;
    const int nl = h.L - h.b;
    int off = 0;
    for (int q = 0; q < nl; ++q) {
        const int l = h.b + q;
        b.coef[q] = h.lv[l].coef64;
        b.cz[q] = h.lv[l].cz;
        for (int a = 0; a < 3; ++a) b.n[q][a] = h.lv[l].n[a];
        b.off_u[q] = off;
        off += (int)h.lv[l].N;
        b.off_f[q] = off;
        off += (int)h.lv[l].N;
        b.off_c[q] = off;
        off += 4 * h.lv[l].n[2];
    }
    b.off_r = off;
    b.nlev = nl;
    b.m = h.m;
    b.nu1 = nu1;
    b.nu2 = nu2;
    b.planar = h.planar ? 1 : 0;
    b.minv = h.minv;
    b.state = state;
    (void)path;
    return b;
}

void add_bottom(Program &pg, Staging &st, const Hierarchy &h, int path, const void *f_top, void *u_top, int nu1,
                int nu2, SolveState *state)
{
    const BottomItem *d = st.put(bottom_item(h, path, f_top, u_top, nu1, nu2, state));
    if (!d) {
        pg.ok = false;
        return;
    }
    Launch L{};
    L.kind = Launch::kBottom;
    L.dbl = path == kF64;
    L.items = d;
    L.lds = h.lds_bytes;
    L.prof = MHS_PROF_BOTTOM;
    L.bytes = (path == kF64 ? 8.0 : 4.0) * 2.0 * (double)h.lv[h.b].N;
    pg.launches.push_back(L);
}

void add_finalize(Program &pg, Staging &st, const double *partials, int n, SolveState *state)
{
    FinalizeItem fi{};
    fi.partials = partials;
    fi.n = n;
    fi.state = state;
    const FinalizeItem *d = st.put(fi);
    if (!d) {
        pg.ok = false;
        return;
    }
    Launch L{};
    L.kind = Launch::kFinalize;
    L.items = d;
    pg.launches.push_back(L);
}

// u += I_z(ec) on level l, whose step to level l+1 halves z only (the
// smoother's fused prolongation assumes halved x and y).
void add_prolong_z(Program &pg, Staging &st, const Hierarchy &h, int l, int path, void *u, const void *ec,
                   SolveState *state)
{
    LevelItem it = level_item(h, l, path);
    const Level &lv = h.lv[l];
    it.u_in = u;
    it.u_out = u;
    it.ec = ec;
    it.state = state;
    it.ntx = ceil_div((lv.n[0] - 2) * (lv.n[1] - 2) * (lv.n[2] - 2), kThreads);
    it.nty = it.ntz = it.kz = 1;
    const LevelItem *d = st.put(it);
    if (!d) {
        pg.ok = false;
        return;
    }
    Launch L{};
    L.kind = Launch::kProlong3Z;
    L.dbl = path == kF64;
    L.items = d;
    L.ntiles = it.ntx;
    L.prof = MHS_PROF_COARSE;
    {
        const double es = path == kF64 ? 8.0 : 4.0;
        L.bytes = es * (2.0 * (double)lv.N + (double)h.lv[l + 1].N);
    }
    pg.launches.push_back(L);
}

// First post-smoothing sweep of level l with the coarse correction ec: fused
// into the sweep, or (after a step that halves z only) added first.
void add_correct_sweep(Program &pg, Staging &st, const Hierarchy &h, int l, int path, void *cur, void *oth,
                       const void *f, const void *ec, SolveState *state, int flags)
{
    if (h.lv[l].keepxy) {
        add_prolong_z(pg, st, h, l, path, cur, ec, state);
        add_sweep(pg, st, h, l, path, cur, oth, f, nullptr, flags, state, nullptr);
    } else {
        add_sweep(pg, st, h, l, path, cur, oth, f, ec, kProlong | flags, state, nullptr);
    }
}

// One V(nu1, nu2) cycle.  Level 0 ping-pongs between a0 (input) and b0; the
// returned pointer is the buffer holding the level-0 result.  With
// `first_norm`, the first sweep also sums the residual of the input iterate
// and a finalize launch follows it (the convergence check of that iterate).
void *add_cycle(Program &pg, Staging &st, const Hierarchy &h, int path, void *a0, void *b0, const void *f0,
                bool first_zero, bool first_norm, int nu1, int nu2, SolveState *state)
{
    const int b = h.b;
    void *cur = a0, *oth = b0;
    // sweeps s0 .. n-1 of level l after the first, ping-pong between c and
    // o; on the 2D hierarchy two per launch (the launch-bound small planes)
    auto more = [&](int l, void *&c, void *&o, const void *f, int s0, int n) {
        for (int s = s0; s < n;) {
            const bool pair = h.planar && s + 1 < n;
            add_sweep(pg, st, h, l, path, c, o, f, nullptr, pair ? kTwoSweeps : 0, state, nullptr);
            std::swap(c, o);
            s += pair ? 2 : 1;
        }
    };
    // the first sweep (flags) and, on the 2D hierarchy, the second with it
    auto pair_first = [&](int n) { return h.planar && n >= 2 ? kTwoSweeps : 0; };
    {
        int flags = pair_first(nu1);
        if (first_zero) flags |= kZeroIn;
        if (first_norm) flags |= kNorm;
        add_sweep(pg, st, h, 0, path, cur, oth, f0, nullptr, flags, state, h.partials);
        std::swap(cur, oth);
        if (first_norm) add_finalize(pg, st, h.partials, h.lv[0].sweep_tiles(), state);
        more(0, cur, oth, f0, (flags & kTwoSweeps) ? 2 : 1, nu1);
    }
    add_restrict(pg, st, h, 0, path, cur, f0, h.lv[1].f[path], state);
    void *lcur[kMaxLevels] = {};
    for (int l = 1; l < b; ++l) {
        const Level &lv = h.lv[l];
        void *c = lv.u[path], *o = lv.t[path];
        // first sweep from a zero guess writes lv.u
        const int fl = kZeroIn | pair_first(nu1);
        add_sweep(pg, st, h, l, path, nullptr, c, lv.f[path], nullptr, fl, state, nullptr);
        more(l, c, o, lv.f[path], (fl & kTwoSweeps) ? 2 : 1, nu1);
        lcur[l] = c;
        add_restrict(pg, st, h, l, path, c, lv.f[path], h.lv[l + 1].f[path], state);
    }
    add_bottom(pg, st, h, path, h.lv[b].f[path], h.lv[b].u[path], nu1, nu2, state);
    const void *ec = h.lv[b].u[path];
    for (int l = b - 1; l >= 1; --l) {
        const Level &lv = h.lv[l];
        void *c = lcur[l];
        void *o = (c == lv.u[path]) ? lv.t[path] : lv.u[path];
        const int fl = pair_first(nu2);
        add_correct_sweep(pg, st, h, l, path, c, o, lv.f[path], ec, state, fl);
        std::swap(c, o);
        more(l, c, o, lv.f[path], fl ? 2 : 1, nu2);
        ec = c;
    }
    {
        const int fl = pair_first(nu2);
        add_correct_sweep(pg, st, h, 0, path, cur, oth, f0, ec, state, fl);
        std::swap(cur, oth);
        more(0, cur, oth, f0, fl ? 2 : 1, nu2);
    }
    return cur;
}

// The FP64 part of one refinement step: u_out = u_in + e (when e is given),
// r32 = -A u_out in FP32, and the norm check of u_out.  The inner FP32
// cycles that produce the next e follow it in the same program.
void add_ir_step(Program &pg, Staging &st, const Hierarchy &h, const double *uin, double *uout, const void *e,
                 float *r32, SolveState *state, bool zero_in)
{
    const Level &l0 = h.lv[0];
    LevelItem it = level_item(h, 0, kF64);
    it.u_in = uin;
    it.u_out = uout;
    it.ec = e;
    it.r_out = r32;
    it.state = state;
    it.partials = h.partials;
    it.ntx = l0.st[0];
    it.nty = l0.ity;
    it.ntz = l0.st[2];
    it.kz = l0.kz;
    const LevelItem *d = st.put(it);
    if (!d) {
        pg.ok = false;
        return;
    }
    Launch L{};
    L.kind = Launch::kIr3;
    L.flags = (e ? 1 : 0) | (zero_in ? 2 : 0);
    L.items = d;
    L.ntiles = l0.ir_tiles();
    L.prof = MHS_PROF_REFINE;
    // read u (not its interior with zero_in) and e, write u and r
    L.bytes = (double)l0.N * ((zero_in ? 0.0 : 8.0) + (e ? 4.0 + 8.0 : 0.0) + 4.0);
    L.pre = true;
    pg.launches.push_back(L);
    add_finalize(pg, st, h.partials, l0.ir_tiles(), state);
}

FieldsItem fields_item(const mhs_plan *p, const mhs_model *model, const double *tab, const double *P, double *Bx,
                       double *By, double *Bz, double *pr, double *rho)
{
    const int nx = p->grid.nx, ny = p->grid.ny, nz = p->grid.nz;
    FieldsItem fi{};
    fi.P = P;
    fi.Bx = Bx;
    fi.By = By;
    fi.Bz = Bz;
    fi.p = pr;
    fi.rho = rho;
    fi.tab = tab;
    fi.alpha = model->alpha;
    fi.mu0 = model->mu0;
    fi.g = model->g;
    fi.dx = p->grid.lx / (nx - 1);
    fi.dy = p->grid.ly / (ny - 1);
    fi.dz = p->grid.lz / (nz - 1);
    fi.nx = nx;
    fi.ny = ny;
    fi.nz = nz;
    fi.ntx = ceil_div(nx - 2, kTX); // interior tiles; edge tiles write the side faces
    fi.nty = ceil_div(ny - 2, kFY);
    fi.kz = chunk(nz, fi.ntx * fi.nty, kKZ, kFieldsTargetGroups);
    fi.ntz = ceil_div(nz, fi.kz);
    fi.tile_base = 0;
    fi.gate = nullptr;
    fi.gate_odd = -1;
    fi.gate_min = 0;
    return fi;
}

int stage_fields(mhs_plan *p, const mhs_model *model, const double *d_P, double *Bx, double *By, double *Bz,
                 double *pr, double *rho, const FieldsItem **d_item, FieldsItem *item)
{
    // the table goes through the staging buffer with the launch items
    const int nz = p->grid.nz;
    const size_t bytes = 4 * (size_t)nz * sizeof(double);
    p->stage.used = (p->stage.used + 63) & ~size_t(63);
    const size_t tab_off = p->stage.used;
    if (tab_off + bytes > p->stage.cap) return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
    double *tab = (double *)(p->stage.host + tab_off);
    std::copy(model->xi, model->xi + nz, tab);
    std::copy(model->dxi, model->dxi + nz, tab + nz);
    std::copy(model->pb, model->pb + nz, tab + 2 * nz);
    std::copy(model->rhob, model->rhob + nz, tab + 3 * nz);
    p->stage.used += bytes;
    *item = fields_item(p, model, (const double *)(p->stage.dev + tab_off), d_P, Bx, By, Bz, pr, rho);
    *d_item = p->stage.put(*item);
    return *d_item ? MHS_OK : fail(MHS_ERR_WORKSPACE, "staging area exhausted");
}

Launch fields_launch(const mhs_plan *p, const FieldsItem *d, const FieldsItem &fi)
{
    Launch L{};
    L.kind = Launch::kFields;
    L.items = d;
    L.ntiles = fi.ntx * fi.nty * fi.ntz;
    L.prof = MHS_PROF_FIELDS;
    L.bytes = 48.0 * (double)p->grid.nx * p->grid.ny * p->grid.nz;
    return L;
}

hipEvent_t prof_event(Profiler &pr)
{
    if (pr.next == pr.pool.size()) {
        hipEvent_t e = nullptr;
        // timing-only events: no system-scope fence (cache writeback) at record
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        pr.pool.push_back(e);
    }
    return pr.pool[pr.next++];
}

// Fold recorded launches into the class totals.  `last` is the index of the
// final cycle/step (the one whose check stopped the solve): its launches
// before the check ran, the rest were skipped by the device-side flag.
int prof_collect(mhs_plan *p, int last)
{
    Profiler &pr = p->prof;
    for (const ProfRecord &r : pr.pending) {
        const bool ran = r.cycle < 0 || r.cycle < last || (r.pre && r.cycle == last);
        if (!ran) continue;
        HIPCHK(hipEventSynchronize(r.end));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, r.start, r.end));
        pr.ms[r.klass] += ms;
        pr.bytes[r.klass] += r.bytes;
        pr.launches[r.klass] += 1;
    }
    pr.pending.clear();
    pr.next = 0;
    return MHS_OK;
}

hipError_t exec_launch(const Launch &L, hipStream_t s)
{
    switch (L.kind) {
    case Launch::kSweep3:
        return launch_sweep3((const LevelItem *)L.items, L.nitems, L.ntiles, L.flags, L.dbl, s);
    case Launch::kSweep2:
        return launch_sweep2((const LevelItem *)L.items, L.nitems, L.ntiles, L.flags, L.dbl, s);
    case Launch::kRestrict3:
        return launch_restrict3((const LevelItem *)L.items, L.nitems, L.ntiles, (L.flags & kRestrictHasF) != 0,
                                (L.flags & kRestrictKeepZ) != 0, L.dbl, s);
    case Launch::kRestrict2:
        return launch_restrict2((const LevelItem *)L.items, L.nitems, L.ntiles, L.dbl, s);
    case Launch::kRestrict3Z:
        return launch_restrict3_z((const LevelItem *)L.items, L.nitems, L.ntiles, (L.flags & kRestrictHasF) != 0,
                                  L.dbl, s);
    case Launch::kProlong3Z:
        return launch_prolong3_z((const LevelItem *)L.items, L.nitems, L.ntiles, L.dbl, s);
    case Launch::kIr3:
        return launch_ir3((const LevelItem *)L.items, L.nitems, L.ntiles, (L.flags & 1) != 0, (L.flags & 2) != 0, s);
    case Launch::kBottom:
        return launch_bottom((const BottomItem *)L.items, L.nitems, L.lds, L.dbl, s);
    case Launch::kFinalize:
        return launch_finalize((const FinalizeItem *)L.items, L.nitems, s);
    case Launch::kCopy:
        return launch_copy(L.src, L.dst, L.n, L.gate, s);
    case Launch::kFields:
        return launch_fields((const FieldsItem *)L.items, L.nitems, L.ntiles, s);
    case Launch::kPrep3:
        return launch_prep3((const PrepItem *)L.items, L.nitems, L.n, s);
    case Launch::kPrep2:
        return launch_prep2((const PrepItem *)L.items, L.nitems, L.n, s);
    case Launch::kGenSweep:
    case Launch::kGenResid:
    case Launch::kGenRestrict:
    case Launch::kGenProlong:
    case Launch::kGenCoarsest:
        return gen_exec(L, s);
    case Launch::kZero:
        return launch_zero(L.dst, (size_t)L.n, s);
    }
    return hipErrorInvalidValue;
}

int run_program(mhs_plan *p, const Program &pg, hipStream_t s, int cycle)
{
    return run_range(p, pg, 0, pg.launches.size(), s, cycle);
}

int run_range(mhs_plan *p, const Program &pg, size_t begin, size_t end, hipStream_t s, int cycle)
{
    Profiler &pr = p->prof;
    for (size_t q = begin; q < end; ++q) {
        const Launch &L = pg.launches[q];
        ProfRecord rec{};
        const bool timed = L.prof >= 0 && ((pr.mask >> L.prof) & 1) != 0;
        if (timed) {
            rec.klass = L.prof;
            rec.cycle = cycle;
            rec.pre = L.pre;
            rec.bytes = L.bytes;
            rec.start = prof_event(pr);
            rec.end = prof_event(pr);
            if (!rec.start || !rec.end) return fail(MHS_ERR_HIP, "event creation failed");
            HIPCHK(hipEventRecord(rec.start, s));
        }
        const hipError_t e = exec_launch(L, s);
        if (e != hipSuccess) return fail(MHS_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
        if (timed) {
            HIPCHK(hipEventRecord(rec.end, s));
            pr.pending.push_back(rec);
        }
    }
    return MHS_OK;
}

bool same_launch(const Launch &a, const Launch &b)
{
    return a.kind == b.kind && a.flags == b.flags && a.dbl == b.dbl && a.items == b.items && a.nitems == b.nitems &&
           a.ntiles == b.ntiles && a.lds == b.lds && a.src == b.src && a.dst == b.dst && a.n == b.n &&
           a.gate == b.gate;
}

// The executable graph of a cycle program: from the plan's cache, else
// captured on the plan's capture stream (nothing runs while capturing).
constexpr size_t kGraphCache = 8;
int cycle_graph(mhs_plan *p, const Program &pg, hipGraphExec_t *out)
{
    *out = nullptr;
    for (CachedGraph &g : p->graphs) {
        if (g.launches.size() != pg.launches.size()) continue;
        bool eq = true;
        for (size_t q = 0; q < pg.launches.size() && eq; ++q) eq = same_launch(g.launches[q], pg.launches[q]);
        if (eq) {
            g.last_use = ++p->graph_clock;
            *out = g.exec;
            return MHS_OK;
        }
    }
    if (!p->cap) HIPCHK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (const Launch &L : pg.launches) {
        le = exec_launch(L, p->cap);
        if (le != hipSuccess) break;
    }
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(p->cap, &graph);
    if (le != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(MHS_ERR_HIP, "cycle capture failed: %s", hipGetErrorString(le != hipSuccess ? le : ee));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(MHS_ERR_HIP, "cycle graph instantiation failed: %s", hipGetErrorString(ie));
    if (p->graphs.size() >= kGraphCache) {
        size_t old = 0;
        for (size_t q = 1; q < p->graphs.size(); ++q)
            if (p->graphs[q].last_use < p->graphs[old].last_use) old = q;
        (void)hipGraphExecDestroy(p->graphs[old].exec);
        p->graphs.erase(p->graphs.begin() + (long)old);
    }
    CachedGraph g;
    g.launches = pg.launches;
    g.exec = exec;
    g.last_use = ++p->graph_clock;
    p->graphs.push_back(std::move(g));
    *out = exec;
    return MHS_OK;
}

int run_cycle(mhs_plan *p, const Program &pg, hipStream_t s, int cycle, bool graph)
{
    if (!graph || !p->graphs_ok || p->prof.mask != 0) return run_program(p, pg, s, cycle);
    hipGraphExec_t exec = nullptr;
    int st = cycle_graph(p, pg, &exec);
    if (st) return st;
    HIPCHK(hipGraphLaunch(exec, s));
    return MHS_OK;
}

int begin_staging(mhs_plan *p)
{
    if (p->stage.inflight) HIPCHK(hipEventSynchronize(p->stage.inflight));
    p->stage.used = 0;
    return MHS_OK;
}

int flush_staging(mhs_plan *p, hipStream_t s)
{
    if (p->stage.used == 0) return MHS_OK;
    HIPCHK(hipMemcpyAsync(p->stage.dev, p->stage.host, p->stage.used, hipMemcpyHostToDevice, s));
    // (a plan without the event waits for its stream before its host
    // staging is reused)
    if (p->stage.inflight) HIPCHK(hipEventRecord(p->stage.inflight, s));
    return MHS_OK;
}

SolveState initial_state(double rtol, int max_iter)
{
    SolveState s{};
    s.rtol = rtol;
    s.max_iter = max_iter;
    return s;
}

int read_state(mhs_plan *p, const SolveState *d_state, SolveState *out, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(p->h_states, d_state, sizeof(SolveState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = p->h_states[0];
    return MHS_OK;
}

// How many more cycles (including the one that only checks) to launch.
int hint_of(const mhs_plan *p, int kind, const mhs_opts *o)
{
    const CycleHint &h = p->last_cycles[kind];
    return h.matches(o) ? h.cycles : 0;
}

void record_cycles(mhs_plan *p, int kind, const mhs_opts *o, const SolveState &ss)
{
    CycleHint &h = p->last_cycles[kind];
    if (ss.done != kConverged) return;
    h.cycles = std::max(0, ss.checks - 1);
    h.rtol = o->rtol;
    h.nu1 = o->nu1;
    h.nu2 = o->nu2;
    h.inner = o->inner_cycles;
}

int next_batch(const SolveState &ss, const mhs_opts *o, int launched, int hint)
{
    const int remaining = o->max_cycles + 1 - launched;
    if (remaining <= 0) return 0;
    if (o->check_every > 0) return std::min(o->check_every, remaining);
    // first batch: as many cycles as the plan's last solve of this kind
    // needed, plus the one that checks; else four
    int want = (launched == 0 && hint > 0) ? hint + 1 : 4;
    if (ss.checks >= 2 && ss.r0 > 0.0 && ss.rnorm > 0.0) {
        const double rel = ss.rnorm / ss.r0;
        const double rate = std::pow(rel, 1.0 / (ss.checks - 1));
        if (rate > 0.0 && rate < 0.95 && o->rtol > 0.0) {
            const double need = std::log(o->rtol / rel) / std::log(rate);
            want = std::max(1, (int)std::ceil(need + 1e-9)) + 1;
        } else {
            want = 8;
        }
    }
    return std::max(1, std::min(want, remaining));
}

int status_of(int32_t done)
{
    switch (done) {
    case kConverged:
        return MHS_OK;
    case kMaxed:
        return MHS_ERR_NO_CONVERGENCE;
    case kDiverged:
        return MHS_ERR_DIVERGED;
    default:
        return MHS_ERR_NO_CONVERGENCE;
    }
}

int set_device(const mhs_plan *p)
{
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != p->device) HIPCHK(hipSetDevice(p->device));
    return MHS_OK;
}

// Drive cycles of `cycle` (each starts with the norm check of the current
// iterate) until the device-side state is no longer running.
// Launches of a program up to and including its convergence check (its first
// finalize; the whole program if it has none).
size_t check_len(const Program &pg)
{
    for (size_t i = 0; i < pg.launches.size(); ++i)
        if (pg.launches[i].kind == Launch::kFinalize) return i + 1;
    return pg.launches.size();
}

// `tail` (optional) enqueues more work after every batch, before its status
// read; `overlap` (optional) runs once on the host after the first two
// programs are enqueued (the device works on them meanwhile; enqueuing a
// whole batch of small launches first would leave the host behind the
// device).
int drive_programs(mhs_plan *p, const std::function<const Program &(int)> &prog, const SolveState *d_state,
                   const mhs_opts *o, int hint, SolveState *out, int *syncs, hipStream_t s,
                   const std::function<int()> *overlap = nullptr, const std::function<int()> *tail = nullptr)
{
    // Each program (cycle or refinement step) starts with the convergence
    // check of the iterate before it.  A batch of nb programs runs the rest
    // of the program whose check ended the previous batch, nb - 1 programs
    // whole and the check of the next one, so the status read after it
    // covers the newest iterate and no launch is issued past a check the
    // host is about to read (graph replays take whole programs).
    const bool graph = o->graph != 0;
    int checked = 0;      // programs whose check has been launched
    size_t resume = 0;    // first launch not yet run of program checked-1 (0: all ran)
    SolveState ss{};
    int st = MHS_OK;
    for (;;) {
        const int nb = next_batch(ss, o, checked, hint);
        if (nb <= 0) break;
        if (resume) {
            const Program &pg = prog(checked - 1);
            if ((st = run_range(p, pg, resume, pg.launches.size(), s, checked - 1))) return st;
            resume = 0;
        }
        for (int q = 0; q < nb; ++q) {
            const int k = checked + q;
            const Program &pg = prog(k);
            const size_t c = check_len(pg);
            if (graph || q + 1 < nb || c == pg.launches.size()) {
                if ((st = run_cycle(p, pg, s, k, graph))) return st;
            } else {
                if ((st = run_range(p, pg, 0, c, s, k))) return st;
                resume = c;
            }
            if (overlap && (q == 1 || q + 1 == nb)) {
                if ((st = (*overlap)())) return st;
                overlap = nullptr;
            }
        }
        checked += nb;
        if (tail && (st = (*tail)())) return st;
        if ((st = read_state(p, d_state, &ss, s))) return st;
        ++*syncs;
        if (ss.done != kRunning) break;
    }
    *out = ss;
    return MHS_OK;
}

int drive(mhs_plan *p, const Program &cycle, const SolveState *d_state, const mhs_opts *o, SolveState *out,
          int *syncs, hipStream_t s, int kind, const std::function<int()> *overlap)
{
    int st = drive_programs(
        p, [&](int) -> const Program & { return cycle; }, d_state, o, hint_of(p, kind, o), out, syncs, s, overlap);
    if (st) return st;
    record_cycles(p, kind, o, *out);
    return prof_collect(p, out->checks - 1);
}

double seconds_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Field recovery requested with an interior solve: launched behind every
// batch of the solve, gated on its convergence, so that a solve whose last
// batch converges as predicted has its fields before its status is read.
struct FieldsReq {
    const mhs_model *model;
    double *Bx, *By, *Bz, *p, *rho;
};
int solve_interior_on(mhs_plan *p, const mhs_model *model, double *d_P, const mhs_opts *o, mhs_info *info,
                      hipStream_t s, std::chrono::steady_clock::time_point t0, const FieldsReq *fr = nullptr);
int solve_boundary_on(mhs_plan *p, const double *d_bz0, double *d_P, const mhs_opts *o, mhs_info *info, hipStream_t s,
                      std::chrono::steady_clock::time_point t0, const std::function<int()> *overlap = nullptr);

} // namespace mhs

// =================================================================================
// C ABI
// =================================================================================
extern "C" {

void mhs_default_opts(mhs_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->precision = MHS_PREC_FP64;
    o->max_cycles = 100;
    o->rtol = 1e-10;
    o->nu1 = 2;
    o->nu2 = 2;
    o->inner_cycles = 3;
    o->warm_start = 0;
    o->check_every = 0;
    o->faces = MHS_FACES_ZERO;
    o->graph = 0;
}

int32_t mhs_version(void) { return 10000; }

const char *mhs_last_error(void) { return g_err.c_str(); }

int mhs_workspace_bytes(const mhs_grid *grid, int32_t precisions, size_t *bytes)
{
    if (!bytes) return fail(MHS_ERR_INVALID_ARG, "bytes is NULL");
    int st = check_grid(grid);
    if (st) return st;
    if (precisions <= 0 || precisions > 7 || (precisions & 3) == 0)
        return fail(MHS_ERR_INVALID_ARG, "precisions must be a mask of 1|2 (at least one), optionally with 4");
    mhs_plan tmp;
    st = geometry(&tmp, grid);
    if (st) return st;
    *bytes = carve_plan(&tmp, nullptr, precisions);
    return MHS_OK;
}

int mhs_request_bytes(const mhs_grid *grid, int32_t precisions, size_t *bytes)
{
    if (!bytes) return fail(MHS_ERR_INVALID_ARG, "bytes is NULL");
    size_t ws = 0;
    const int st = mhs_workspace_bytes(grid, precisions, &ws);
    if (st) return st;
    const size_t n = (size_t)grid->nx * grid->ny * grid->nz;
    *bytes = ws + 6 * sizeof(double) * n + sizeof(double) * (size_t)grid->nx * grid->ny;
    return MHS_OK;
}

int mhs_check_model(const mhs_grid *grid, const mhs_model *model, double *lambda_min, int32_t *levels)
{
    int st = check_grid(grid);
    if (st) return st;
    mhs_plan tmp;
    if ((st = geometry(&tmp, grid))) return st;
    if ((st = validate_model(&tmp, model, false))) return st;
    int depth = 0;
    if ((st = model_depth(tmp.h3, *grid, model, &depth, lambda_min))) return st;
    if ((st = set_depth(tmp.h3, depth))) return st;
    if (levels) *levels = depth;
    return MHS_OK;
}

int mhs_plan_create(const mhs_grid *grid, int32_t precisions, void *d_ws, size_t ws_bytes, mhs_plan **out)
{
    if (!out) return fail(MHS_ERR_INVALID_ARG, "plan output is NULL");
    *out = nullptr;
    size_t need = 0;
    int st = mhs_workspace_bytes(grid, precisions, &need);
    if (st) return st;
    if (!d_ws || ((uintptr_t)d_ws % kAlign) != 0)
        return fail(MHS_ERR_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < need) return fail(MHS_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    mhs_plan *p = new mhs_plan();
    p->precisions = precisions;
    HIPCHK(hipGetDevice(&p->device));
    st = geometry(p, grid);
    if (st) {
        delete p;
        return st;
    }
    p->ws = (char *)d_ws;
    p->ws_bytes = ws_bytes;
    carve_plan(p, p->ws, precisions);
    if (hipHostMalloc((void **)&p->stage.host, kStagingBytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&p->h_states, 4 * sizeof(SolveState), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&p->stage.inflight, hipEventDisableTiming) != hipSuccess) {
        mhs_plan_destroy(p);
        return fail(MHS_ERR_HIP, "pinned host allocation failed");
    }
    // boundary nodes of every coarse array must read as zero
    if (hipMemset(d_ws, 0, need - kAlign) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        mhs_plan_destroy(p);
        return fail(MHS_ERR_HIP, "workspace clear failed");
    }
    hipStream_t s0 = nullptr;
    st = upload_planar(p, s0);
    if (st) {
        mhs_plan_destroy(p);
        return st;
    }
    *out = p;
    return MHS_OK;
}

int mhs_plan_destroy(mhs_plan *p)
{
    if (!p) return MHS_OK;
    if (p->stage.inflight) {
        (void)hipEventSynchronize(p->stage.inflight);
        (void)hipEventDestroy(p->stage.inflight);
    }
    for (hipEvent_t e : p->prof.pool) (void)hipEventDestroy(e);
    if (p->stage.host) (void)hipHostFree(p->stage.host);
    if (p->h_states) (void)hipHostFree(p->h_states);
    for (mhs::CachedGraph &g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    delete p;
    return MHS_OK;
}

int mhs_plan_levels(const mhs_plan *p, int32_t space, int32_t *nlevels)
{
    if (!p || !nlevels) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    if (space != 2 && space != 3) return fail(MHS_ERR_INVALID_ARG, "space must be 2 or 3");
    *nlevels = space == 3 ? p->h3.L : p->h2.L;
    return MHS_OK;
}

int mhs_plan_level_dims(const mhs_plan *p, int32_t space, int32_t level, int32_t *nx, int32_t *ny, int32_t *nz)
{
    if (!p || !nx || !ny || !nz) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    if (space != 2 && space != 3) return fail(MHS_ERR_INVALID_ARG, "space must be 2 or 3");
    const Hierarchy &h = space == 3 ? p->h3 : p->h2;
    if (level < 0 || level >= h.L) return fail(MHS_ERR_INVALID_ARG, "level out of range");
    *nx = h.lv[level].n[0];
    *ny = h.lv[level].n[1];
    *nz = h.lv[level].n[2];
    return MHS_OK;
}

int mhs_plan_bottom_level(const mhs_plan *p, int32_t space, int32_t *level)
{
    if (!p || !level) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    if (space != 2 && space != 3) return fail(MHS_ERR_INVALID_ARG, "space must be 2 or 3");
    *level = space == 3 ? p->h3.b : p->h2.b;
    return MHS_OK;
}

int mhs_solve_boundary(mhs_plan *p, const double *d_bz0, double *d_P, const mhs_opts *o, mhs_info *info,
                       void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!p || !d_bz0 || !d_P) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    int st = validate_opts(o);
    if (st) return st;
    if ((st = set_device(p))) return st;
    return solve_boundary_on(p, d_bz0, d_P, o, info, (hipStream_t)stream, t0);
}

} // extern "C"

namespace mhs {

// The base solve on a plan whose device is current, with validated options.
int solve_boundary_on(mhs_plan *p, const double *d_bz0, double *d_P, const mhs_opts *o, mhs_info *info, hipStream_t s,
                      std::chrono::steady_clock::time_point t0, const std::function<int()> *overlap)
{
    int st = MHS_OK;
    Hierarchy &h = p->h2;
    if ((st = begin_staging(p))) return st;
    SolveState *d_state = (SolveState *)p->stage.put(initial_state(o->rtol, o->max_cycles));
    PrepItem pi{};
    pi.P = d_P;
    pi.twin = (double *)h.lv[0].t[kF64];
    pi.bz0 = d_bz0;
    pi.f2 = (double *)h.lv[0].f[kF64];
    pi.nx = p->grid.nx;
    pi.ny = p->grid.ny;
    pi.nz = 1;
    pi.warm = o->warm_start;
    pi.faces = o->faces;
    pi.n = (int64_t)p->grid.nx * p->grid.ny;
    pi.base = 0;
    const PrepItem *d_prep = p->stage.put(pi);
    Program cyc;
    void *res = add_cycle(cyc, p->stage, h, kF64, d_P, h.lv[0].t[kF64], h.lv[0].f[kF64], false, true, o->nu1,
                          o->nu2, d_state);
    if (res != (void *)d_P) {
        Launch c{};
        c.kind = Launch::kCopy;
        c.src = (const double *)res;
        c.dst = d_P;
        c.n = (int64_t)p->grid.nx * p->grid.ny;
        c.gate = d_state;
        cyc.launches.push_back(c);
    }
    if (!cyc.ok || !d_state || !d_prep) return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
    if ((st = flush_staging(p, s))) return st;
    HIPCHK(launch_prep2(d_prep, 1, pi.n, s));
    SolveState fin{};
    int syncs = 0;
    if ((st = drive(p, cyc, d_state, o, &fin, &syncs, s, kSolve2D, overlap))) return st;
    const int status = status_of(fin.done);
    if (info) {
        info->status = status;
        info->cycles = std::max(0, fin.checks - 1);
        info->inner_cycles = 0;
        info->host_syncs = syncs;
        info->r0 = fin.r0;
        info->rel_residual = fin.r0 > 0 ? fin.rnorm / fin.r0 : 0.0;
        info->seconds = seconds_since(t0);
    }
    if (status != MHS_OK)
        return fail(status, "lower-boundary solve stopped after %d cycles (relative residual %g)", fin.checks - 1,
                    fin.r0 > 0 ? fin.rnorm / fin.r0 : 0.0);
    return MHS_OK;
}

} // namespace mhs

extern "C" {

int mhs_solve_interior(mhs_plan *p, const mhs_model *model, double *d_P, const mhs_opts *o, mhs_info *info,
                       void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!p || !d_P) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    int st = validate_opts(o);
    if (st) return st;
    if ((st = validate_model(p, model, false))) return st;
    if (!(p->precisions & o->precision))
        return fail(MHS_ERR_UNSUPPORTED, "plan was not created for precision %d", o->precision);
    if ((st = set_device(p))) return st;
    return solve_interior_on(p, model, d_P, o, info, (hipStream_t)stream, t0);
}

int mhs_solve_equilibrium(mhs_plan *p, const mhs_model *model, const double *d_bz0, double *d_P, double *d_Bx,
                          double *d_By, double *d_Bz, double *d_p, double *d_rho, const mhs_opts *o2,
                          const mhs_opts *o3, mhs_info *info2, mhs_info *info3, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!p || !d_bz0 || !d_P) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    const int nf = (d_Bx != nullptr) + (d_By != nullptr) + (d_Bz != nullptr) + (d_p != nullptr) + (d_rho != nullptr);
    if (nf != 0 && nf != 5) return fail(MHS_ERR_INVALID_ARG, "field outputs: all five or none");
    int st = validate_opts(o2);
    if (st) return st;
    if ((st = validate_opts(o3))) return st;
    if ((st = validate_model(p, model, nf == 5))) return st;
    if (!(p->precisions & o3->precision))
        return fail(MHS_ERR_UNSUPPORTED, "plan was not created for precision %d", o3->precision);
    if ((st = set_device(p))) return st;
    hipStream_t s = (hipStream_t)stream;
    // the model's 3D tables are prepared on the host while the first batch
    // of base cycles runs
    ModelUpload up;
    int prep_st = MHS_OK;
    bool prepared = false;
    const std::function<int()> prep = [&]() -> int {
        prep_st = prepare_model(p, model, up);
        prepared = prep_st == MHS_OK;
        return MHS_OK;
    };
    st = solve_boundary_on(p, d_bz0, d_P, o2, info2, s, t0, &prep);
    if (!st && !prepared && prep_st == MHS_OK) prep_st = prepare_model(p, model, up); // the hook did not run
    if (st || prep_st) {
        if (prepared && !up.parts.empty()) invalidate_model(p); // the tables never reach the device
        return st ? st : prep_st;
    }
    for (const ModelUpload::Part &q : up.parts)
        HIPCHK(hipMemcpyAsync(q.dst, up.data.data() + q.off, q.bytes, hipMemcpyHostToDevice, s));
    // pageable source: the copy has consumed it before `up` goes away
    if (!up.parts.empty()) HIPCHK(hipStreamSynchronize(s));
    const FieldsReq fr{model, d_Bx, d_By, d_Bz, d_p, d_rho};
    return solve_interior_on(p, model, d_P, o3, info3, s, std::chrono::steady_clock::now(), nf ? &fr : nullptr);
}

} // extern "C"

namespace mhs {

// The interior solve on a validated plan whose device is current.
int solve_interior_on(mhs_plan *p, const mhs_model *model, double *d_P, const mhs_opts *o, mhs_info *info,
                      hipStream_t s, std::chrono::steady_clock::time_point t0, const FieldsReq *fr)
{
    int st = MHS_OK;
    Hierarchy &h = p->h3;
    if ((st = upload_model(p, model, s))) return st;
    if ((st = begin_staging(p))) return st;
    const bool mixed = o->precision == MHS_PREC_MIXED;
    SolveState *d_state = (SolveState *)p->stage.put(initial_state(o->rtol, o->max_cycles));
    double *T0 = (double *)h.lv[0].t[kF64];
    const int64_t N = (int64_t)h.lv[0].N;
    // mixed path: when the plan's last solve of this kind took an odd number
    // of refinement steps, a cold start begins from the twin, so that the
    // same count ends in P with no copy
    const int hint = mixed ? hint_of(p, kSolve3DMixed, o) : 0;
    const bool swap = mixed && !o->warm_start && (hint & 1);
    // mixed cold start: no interior is zeroed; the first two refinement
    // steps read the start iterate's interior as zero (its boundary nodes
    // only), and a solve that stops at step 0 zeroes P's interior after
    const bool keep = mixed && !o->warm_start;
    PrepItem pi{};
    pi.P = d_P;
    pi.twin = T0;
    pi.nx = p->grid.nx;
    pi.ny = p->grid.ny;
    pi.nz = p->grid.nz;
    pi.warm = o->warm_start;
    pi.faces = o->faces;
    pi.swap = swap ? 1 : 0;
    pi.keep = keep ? 1 : 0;
    pi.n = keep ? prep3_faces(pi.nx, pi.ny, pi.nz) : N;
    const PrepItem *d_prep = p->stage.put(pi);
    PrepItem pz = pi; // P's interior zeroed, faces as above
    pz.swap = 0;
    pz.keep = 0;
    pz.n = N;
    const PrepItem *d_zero = keep ? p->stage.put(pz) : nullptr;
    SolveState fin{};
    int syncs = 0;
    int inner_total = 0;
    // field recovery (fr): an item gated on convergence with P holding the
    // iterate, launched behind every batch, and an ungated one for a solve
    // whose iterate ends in the twin (run after the copy)
    const FieldsItem *d_fgated = nullptr, *d_fplain = nullptr;
    FieldsItem fitem{};
    bool fields_done = false;
    auto stage_fields_pair = [&](const SolveState *gate, int gate_odd, int gate_min) -> int {
        int e = stage_fields(p, fr->model, d_P, fr->Bx, fr->By, fr->Bz, fr->p, fr->rho, &d_fplain, &fitem);
        if (e) return e;
        FieldsItem g = fitem;
        g.gate = gate;
        g.gate_odd = gate_odd;
        g.gate_min = gate_min;
        d_fgated = p->stage.put(g);
        return d_fgated ? MHS_OK : fail(MHS_ERR_WORKSPACE, "staging area exhausted");
    };
    const std::function<int()> gated_fields = [&]() -> int {
        Program pg;
        Launch L = fields_launch(p, d_fgated, fitem);
        L.prof = -1; // mostly a launch that exits at once: not timed
        pg.launches.push_back(L);
        return run_program(p, pg, s);
    };
    if (!mixed) {
        Program cyc;
        void *res = add_cycle(cyc, p->stage, h, kF64, d_P, T0, nullptr, false, true, o->nu1, o->nu2, d_state);
        if (res != (void *)d_P) {
            Launch c{};
            c.kind = Launch::kCopy;
            c.src = (const double *)res;
            c.dst = d_P;
            c.n = N;
            c.gate = d_state;
            cyc.launches.push_back(c);
        }
        if (!cyc.ok || !d_state || !d_prep) return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
        if (fr && (st = stage_fields_pair(d_state, -1, 0))) return st;
        if ((st = flush_staging(p, s))) return st;
        HIPCHK(launch_prep3(d_prep, 1, prep3_threads(pi.n), s));
        if ((st = drive_programs(
                 p, [&](int) -> const Program & { return cyc; }, d_state, o, hint_of(p, kSolve3D64, o), &fin, &syncs,
                 s, nullptr, fr ? &gated_fields : nullptr)))
            return st;
        record_cycles(p, kSolve3D64, o, fin);
        if ((st = prof_collect(p, fin.checks - 1))) return st;
        // P holds the iterate of every checked cycle: the gated recovery ran
        fields_done = true;
    } else {
        // FP64 iterative refinement around FP32 V-cycles.  Step 0 only
        // computes r = -A U; step s >= 1 applies the previous correction
        // (U -> V for odd s, V -> U for even s) and recomputes r.  U is P
        // and V its twin, or the other way round (`swap`).
        double *U = swap ? T0 : d_P, *V = swap ? d_P : T0;
        const Level &l0 = h.lv[0];
        float *r32 = (float *)l0.f[kF32];
        // inner cycles: locate the final correction buffer
        Program inner;
        void *ebuf = nullptr;
        for (int c = 0; c < o->inner_cycles; ++c) {
            void *a = c == 0 ? l0.u[kF32] : ebuf;
            void *bb = (a == l0.u[kF32]) ? l0.t[kF32] : l0.u[kF32];
            ebuf = add_cycle(inner, p->stage, h, kF32, a, bb, r32, c == 0, false, o->nu1, o->nu2, d_state);
        }
        Program first, second, odd, even;
        add_ir_step(first, p->stage, h, U, nullptr, nullptr, r32, d_state, keep);
        if (keep) add_ir_step(second, p->stage, h, U, V, ebuf, r32, d_state, true);
        add_ir_step(odd, p->stage, h, U, V, ebuf, r32, d_state);
        add_ir_step(even, p->stage, h, V, U, ebuf, r32, d_state);
        for (Program *pg : {&first, &second, &odd, &even})
            if (pg != &second || keep) pg->launches.insert(pg->launches.end(), inner.launches.begin(), inner.launches.end());
        if (!first.ok || !second.ok || !odd.ok || !even.ok || !inner.ok || !d_state || !d_prep || (keep && !d_zero))
            return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
        // P holds the iterate after an odd count with swap, an even one
        // without (after a cold start, from step 1 on)
        if (fr && (st = stage_fields_pair(d_state, swap ? 1 : 0, keep ? 1 : 0))) return st;
        if ((st = flush_staging(p, s))) return st;
        HIPCHK(launch_prep3(d_prep, 1, prep3_threads(pi.n), s));
        SolveState ss{};
        if ((st = drive_programs(
                 p,
                 [&](int step) -> const Program & {
                     return step == 0 ? first : (step == 1 && keep) ? second : ((step & 1) ? odd : even);
                 },
                 d_state, o, hint, &ss, &syncs, s, nullptr, fr ? &gated_fields : nullptr)))
            return st;
        fin = ss;
        record_cycles(p, kSolve3DMixed, o, ss);
        if ((st = prof_collect(p, fin.checks - 1))) return st;
        const int steps = std::max(0, fin.checks - 1);
        inner_total = steps * o->inner_cycles;
        // the iterate ends in V after an odd step count, else in U; when
        // that is the twin, the copy is stream-ordered like the rest of the
        // solve's work.  A cold start stopped at step 0 never wrote an
        // interior: P's is zeroed.
        if (keep && steps == 0)
            HIPCHK(launch_prep3(d_zero, 1, prep3_threads(N), s));
        else if (((steps & 1) ? V : U) == T0)
            HIPCHK(launch_copy(T0, d_P, N, nullptr, s));
        else
            fields_done = true;
    }
    const int status = status_of(fin.done);
    if (fr && status == MHS_OK && !fields_done) {
        Program pg;
        pg.launches.push_back(fields_launch(p, d_fplain, fitem));
        if ((st = run_program(p, pg, s))) return st;
    }
    if (info) {
        info->status = status;
        info->cycles = std::max(0, fin.checks - 1);
        info->inner_cycles = inner_total;
        info->host_syncs = syncs;
        info->r0 = fin.r0;
        info->rel_residual = fin.r0 > 0 ? fin.rnorm / fin.r0 : 0.0;
        info->seconds = seconds_since(t0);
    }
    if (status != MHS_OK)
        return fail(status, "interior solve stopped after %d cycles (relative residual %g)", fin.checks - 1,
                    fin.r0 > 0 ? fin.rnorm / fin.r0 : 0.0);
    return MHS_OK;
}

} // namespace mhs

extern "C" {

int mhs_fields(mhs_plan *p, const mhs_model *model, const double *d_P, double *d_Bx, double *d_By, double *d_Bz,
               double *d_p, double *d_rho, void *stream)
{
    if (!p || !d_P || !d_Bx || !d_By || !d_Bz || !d_p || !d_rho) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    int st = validate_model(p, model, true);
    if (st) return st;
    if ((st = set_device(p))) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = begin_staging(p))) return st;
    const FieldsItem *d = nullptr;
    FieldsItem fi{};
    if ((st = stage_fields(p, model, d_P, d_Bx, d_By, d_Bz, d_p, d_rho, &d, &fi))) return st;
    if ((st = flush_staging(p, s))) return st;
    Program pg;
    pg.launches.push_back(fields_launch(p, d, fi));
    return run_program(p, pg, s);
}

int mhs_diagnostics(mhs_plan *p, const mhs_model *model, const double *d_Bx, const double *d_By,
                    const double *d_Bz, const double *d_p, const double *d_rho, double *d_jx, double *d_jy,
                    double *d_jz, double *d_fres, double *d_divb, void *stream)
{
    if (!p || !model || !d_Bx || !d_By || !d_Bz || !d_p || !d_rho || !d_jx || !d_jy || !d_jz || !d_fres || !d_divb)
        return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    if (!(model->mu0 > 0.0) || !std::isfinite(model->mu0) || !std::isfinite(model->g))
        return fail(MHS_ERR_INVALID_ARG, "mu0 must be positive and g finite");
    int st = set_device(p);
    if (st) return st;
    const int nx = p->grid.nx, ny = p->grid.ny, nz = p->grid.nz;
    DiagItem it{};
    it.Bx = d_Bx;
    it.By = d_By;
    it.Bz = d_Bz;
    it.p = d_p;
    it.rho = d_rho;
    it.jx = d_jx;
    it.jy = d_jy;
    it.jz = d_jz;
    it.fres = d_fres;
    it.divb = d_divb;
    it.mu0 = model->mu0;
    it.g = model->g;
    it.dx = p->grid.lx / (nx - 1);
    it.dy = p->grid.ly / (ny - 1);
    it.dz = p->grid.lz / (nz - 1);
    it.nx = nx;
    it.ny = ny;
    it.nz = nz;
    it.kz = chunk(nz, ceil_div(nx, 64) * ceil_div(ny, 4), 64, kFieldsTargetGroups);
    hipStream_t s = (hipStream_t)stream;
    Profiler &pr = p->prof;
    const bool timed = ((pr.mask >> MHS_PROF_DIAG) & 1) != 0;
    ProfRecord rec{};
    if (timed) {
        rec.klass = MHS_PROF_DIAG;
        rec.cycle = -1;
        rec.bytes = 80.0 * (double)nx * ny * nz;
        rec.start = prof_event(pr);
        rec.end = prof_event(pr);
        if (!rec.start || !rec.end) return fail(MHS_ERR_HIP, "event creation failed");
        HIPCHK(hipEventRecord(rec.start, s));
    }
    const hipError_t e = launch_diag(it, s);
    if (e != hipSuccess) return fail(MHS_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    if (timed) {
        HIPCHK(hipEventRecord(rec.end, s));
        pr.pending.push_back(rec);
    }
    return MHS_OK;
}

int mhs_trace_field_lines(mhs_plan *p, const double *d_Bx, const double *d_By, const double *d_Bz,
                          const double *d_seeds, int32_t nlines, double ds, int32_t max_steps, double bmin,
                          double *d_points, int32_t *d_count, int32_t *d_status, void *stream)
{
    if (!p) return fail(MHS_ERR_INVALID_ARG, "plan is NULL");
    if (nlines < 0 || max_steps < 0) return fail(MHS_ERR_INVALID_ARG, "nlines and max_steps must be >= 0");
    if (!(ds != 0.0) || !std::isfinite(ds)) return fail(MHS_ERR_INVALID_ARG, "ds must be finite and nonzero");
    if (!(bmin >= 0.0) || !std::isfinite(bmin)) return fail(MHS_ERR_INVALID_ARG, "bmin must be finite and >= 0");
    if (nlines == 0) return MHS_OK;
    if (!d_Bx || !d_By || !d_Bz || !d_seeds || !d_points || !d_count || !d_status)
        return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    int st = set_device(p);
    if (st) return st;
    TraceItem it{};
    it.Bx = d_Bx;
    it.By = d_By;
    it.Bz = d_Bz;
    it.seeds = d_seeds;
    it.points = d_points;
    it.count = d_count;
    it.status = d_status;
    it.lx = p->grid.lx;
    it.ly = p->grid.ly;
    it.lz = p->grid.lz;
    it.dx = p->grid.lx / (p->grid.nx - 1);
    it.dy = p->grid.ly / (p->grid.ny - 1);
    it.dz = p->grid.lz / (p->grid.nz - 1);
    it.ds = ds;
    it.bmin = bmin;
    it.nx = p->grid.nx;
    it.ny = p->grid.ny;
    it.nz = p->grid.nz;
    it.nlines = nlines;
    it.max_steps = max_steps;
    hipStream_t s = (hipStream_t)stream;
    Profiler &pr = p->prof;
    const bool timed = ((pr.mask >> MHS_PROF_TRACE) & 1) != 0;
    ProfRecord rec{};
    if (timed) {
        rec.klass = MHS_PROF_TRACE;
        rec.cycle = -1;
        rec.bytes = 0.0; // gathers through the caches: no compulsory-traffic model
        rec.start = prof_event(pr);
        rec.end = prof_event(pr);
        if (!rec.start || !rec.end) return fail(MHS_ERR_HIP, "event creation failed");
        HIPCHK(hipEventRecord(rec.start, s));
    }
    const hipError_t e = launch_trace(it, s);
    if (e != hipSuccess) return fail(MHS_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    if (timed) {
        HIPCHK(hipEventRecord(rec.end, s));
        pr.pending.push_back(rec);
    }
    return MHS_OK;
}

int mhs_profile_enable(mhs_plan *p, int32_t class_mask)
{
    if (!p) return fail(MHS_ERR_INVALID_ARG, "plan is NULL");
    if (class_mask < 0 || class_mask > MHS_PROF_ALL) return fail(MHS_ERR_INVALID_ARG, "bad class mask");
    p->prof.mask = class_mask;
    return MHS_OK;
}

int mhs_profile_read(mhs_plan *p, int32_t klass, double *total_ms, int64_t *launches, double *bytes,
                     int32_t reset)
{
    if (!p || klass < 0 || klass >= MHS_PROF_NCLASS) return fail(MHS_ERR_INVALID_ARG, "bad plan or class");
    int st = prof_collect(p, -1 + (1 << 30)); // anything still pending was launched by an asynchronous call
    if (st) return st;
    if (total_ms) *total_ms = p->prof.ms[klass];
    if (launches) *launches = p->prof.launches[klass];
    if (bytes) *bytes = p->prof.bytes[klass];
    if (reset) {
        for (int k = 0; k < MHS_PROF_NCLASS; ++k) {
            p->prof.ms[k] = 0.0;
            p->prof.bytes[k] = 0.0;
            p->prof.launches[k] = 0;
        }
    }
    return MHS_OK;
}

} // extern "C"

// ---- stage entry points -----------------------------------------------------------
namespace {

int stage_common(mhs_plan *p, const mhs_model *model, int space, int level, int precision, Hierarchy **hh,
                 int *path, hipStream_t s)
{
    if (!p) return fail(MHS_ERR_INVALID_ARG, "plan is NULL");
    if (space != 2 && space != 3) return fail(MHS_ERR_INVALID_ARG, "space must be 2 or 3");
    if (precision != MHS_PREC_FP64 && precision != MHS_PREC_MIXED)
        return fail(MHS_ERR_INVALID_ARG, "precision must be MHS_PREC_FP64 or MHS_PREC_MIXED");
    Hierarchy &h = space == 3 ? p->h3 : p->h2;
    if (level < 0 || level >= h.L) return fail(MHS_ERR_INVALID_ARG, "level out of range");
    if (space == 2 && precision != MHS_PREC_FP64) return fail(MHS_ERR_UNSUPPORTED, "2D stages are FP64 only");
    if (space == 3 && !(p->precisions & precision))
        return fail(MHS_ERR_UNSUPPORTED, "plan was not created for precision %d", precision);
    int st = set_device(p);
    if (st) return st;
    if (space == 3) {
        if ((st = validate_model(p, model, false))) return st;
        if ((st = upload_model(p, model, s))) return st;
    }
    *hh = &h;
    *path = precision == MHS_PREC_FP64 ? kF64 : kF32;
    return MHS_OK;
}

// the level's ping-pong twin for stage calls
void *stage_twin(Hierarchy &h, int level, int path) { return h.lv[level].t[path]; }

// Stage calls borrow a solver twin as scratch; the solver relies on the
// boundary nodes of every twin being zero (the level-0 FP64 twin is reset by
// each interior solve), so clear the borrowed buffer afterwards.
int release_twin(Hierarchy &h, int level, int path, hipStream_t s)
{
    const size_t bytes = h.lv[level].N * (path == kF64 ? 8 : 4);
    HIPCHK(hipMemsetAsync(h.lv[level].t[path], 0, bytes, s));
    return MHS_OK;
}

} // namespace

extern "C" {

int mhs_stage_smooth(mhs_plan *p, const mhs_model *model, int32_t space, int32_t level, int32_t precision,
                     void *d_u, const void *d_f, int32_t nsweeps, int32_t zero_guess, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Hierarchy *h = nullptr;
    int path = 0;
    int st = stage_common(p, model, space, level, precision, &h, &path, s);
    if (st) return st;
    if (!d_u || nsweeps < 1 || (zero_guess != 0 && zero_guess != 1))
        return fail(MHS_ERR_INVALID_ARG, "bad u, nsweeps or zero_guess");
    if (zero_guess && !d_f) return fail(MHS_ERR_INVALID_ARG, "a sweep from a zero guess needs f");
    void *tw = stage_twin(*h, level, path);
    if (!tw || level >= h->b) return fail(MHS_ERR_UNSUPPORTED, "level %d is handled by the bottom solver", level);
    if (path == kF32 && level == 0) tw = h->lv[0].t[kF32];
    const size_t es = path == kF64 ? 8 : 4;
    const size_t bytes = h->lv[level].N * es;
    HIPCHK(hipMemcpyAsync(tw, d_u, bytes, hipMemcpyDeviceToDevice, s));
    if ((st = begin_staging(p))) return st;
    Program pg;
    void *cur = d_u, *oth = tw;
    // as in the cycles: on the 2D hierarchy two sweeps per launch
    for (int q = 0; q < nsweeps;) {
        const bool zero = q == 0 && zero_guess;
        const bool pair = h->planar && q + 1 < nsweeps;
        add_sweep(pg, p->stage, *h, level, path, zero ? nullptr : cur, oth, d_f, nullptr,
                  (zero ? kZeroIn : 0) | (pair ? kTwoSweeps : 0), nullptr, nullptr);
        std::swap(cur, oth);
        q += pair ? 2 : 1;
    }
    if (!pg.ok) return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
    if ((st = flush_staging(p, s))) return st;
    if ((st = run_program(p, pg, s))) return st;
    if (cur != d_u) HIPCHK(hipMemcpyAsync(d_u, cur, bytes, hipMemcpyDeviceToDevice, s));
    return release_twin(*h, level, path, s);
}

int mhs_stage_restrict(mhs_plan *p, const mhs_model *model, int32_t space, int32_t level, int32_t precision,
                       const void *d_u, const void *d_f, void *d_fc, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Hierarchy *h = nullptr;
    int path = 0;
    int st = stage_common(p, model, space, level, precision, &h, &path, s);
    if (st) return st;
    if (!d_u || !d_fc || level + 1 >= h->L) return fail(MHS_ERR_INVALID_ARG, "bad arrays or level");
    if (space == 2 && !d_f) return fail(MHS_ERR_INVALID_ARG, "2D restriction needs f");
    if ((st = begin_staging(p))) return st;
    Program pg;
    add_restrict(pg, p->stage, *h, level, path, d_u, d_f, d_fc, nullptr);
    if (!pg.ok) return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
    if ((st = flush_staging(p, s))) return st;
    return run_program(p, pg, s);
}

int mhs_stage_correct_smooth(mhs_plan *p, const mhs_model *model, int32_t space, int32_t level, int32_t precision,
                             void *d_u, const void *d_f, const void *d_ec, int32_t nsweeps, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Hierarchy *h = nullptr;
    int path = 0;
    int st = stage_common(p, model, space, level, precision, &h, &path, s);
    if (st) return st;
    if (!d_u || !d_ec || level + 1 >= h->L || nsweeps < 1) return fail(MHS_ERR_INVALID_ARG, "bad arrays, level or nsweeps");
    void *tw = stage_twin(*h, level, path);
    if (!tw || level >= h->b) return fail(MHS_ERR_UNSUPPORTED, "level %d is handled by the bottom solver", level);
    if (path == kF32 && level == 0) tw = h->lv[0].t[kF32];
    const size_t bytes = h->lv[level].N * (path == kF64 ? 8 : 4);
    HIPCHK(hipMemcpyAsync(tw, d_u, bytes, hipMemcpyDeviceToDevice, s));
    if ((st = begin_staging(p))) return st;
    Program pg;
    void *cur = d_u, *oth = tw;
    // as in the cycles: on the 2D hierarchy two sweeps per launch
    const bool pair0 = h->planar && nsweeps >= 2;
    add_correct_sweep(pg, p->stage, *h, level, path, cur, oth, d_f, d_ec, nullptr, pair0 ? kTwoSweeps : 0);
    std::swap(cur, oth);
    for (int q = pair0 ? 2 : 1; q < nsweeps;) {
        const bool pair = h->planar && q + 1 < nsweeps;
        add_sweep(pg, p->stage, *h, level, path, cur, oth, d_f, nullptr, pair ? kTwoSweeps : 0, nullptr, nullptr);
        std::swap(cur, oth);
        q += pair ? 2 : 1;
    }
    if (!pg.ok) return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
    if ((st = flush_staging(p, s))) return st;
    if ((st = run_program(p, pg, s))) return st;
    if (cur != d_u) HIPCHK(hipMemcpyAsync(d_u, cur, bytes, hipMemcpyDeviceToDevice, s));
    return release_twin(*h, level, path, s);
}

int mhs_stage_bottom(mhs_plan *p, const mhs_model *model, int32_t space, int32_t precision, void *d_u,
                     const void *d_f, int32_t nu1, int32_t nu2, int32_t *bottom_level, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Hierarchy *h = nullptr;
    int path = 0;
    int st = stage_common(p, model, space, 0, precision, &h, &path, s);
    if (st) return st;
    if (!d_u || !d_f || nu1 < 1 || nu2 < 1) return fail(MHS_ERR_INVALID_ARG, "bad arguments");
    if (bottom_level) *bottom_level = h->b;
    if ((st = begin_staging(p))) return st;
    Program pg;
    add_bottom(pg, p->stage, *h, path, d_f, d_u, nu1, nu2, nullptr);
    if (!pg.ok) return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
    if ((st = flush_staging(p, s))) return st;
    return run_program(p, pg, s);
}

int mhs_stage_residual_norm(mhs_plan *p, const mhs_model *model, int32_t space, int32_t level, int32_t precision,
                            const void *d_u, const void *d_f, double *norm, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Hierarchy *h = nullptr;
    int path = 0;
    int st = stage_common(p, model, space, level, precision, &h, &path, s);
    if (st) return st;
    if (!d_u || !norm) return fail(MHS_ERR_INVALID_ARG, "bad arguments");
    void *tw = stage_twin(*h, level, path);
    if (!tw || level >= h->b) return fail(MHS_ERR_UNSUPPORTED, "level %d is handled by the bottom solver", level);
    if (h->lv[level].sweep_tiles() > p->scratch_npart) return fail(MHS_ERR_WORKSPACE, "scratch too small");
    if ((st = begin_staging(p))) return st;
    SolveState *d_state = (SolveState *)p->stage.put(initial_state(0.0, 0));
    Program pg;
    add_sweep(pg, p->stage, *h, level, path, d_u, tw, d_f, nullptr, kNorm, nullptr, p->d_scratch_norm);
    add_finalize(pg, p->stage, p->d_scratch_norm, h->lv[level].sweep_tiles(), d_state);
    if (!pg.ok || !d_state) return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
    if ((st = flush_staging(p, s))) return st;
    if ((st = run_program(p, pg, s))) return st;
    if ((st = release_twin(*h, level, path, s))) return st;
    SolveState ss{};
    if ((st = read_state(p, d_state, &ss, s))) return st;
    *norm = ss.rnorm;
    return MHS_OK;
}

} // extern "C"

// =================================================================================
// Interior solve over a scratch array the library owns (no allocation per call)
// =================================================================================
namespace {

// The largest workspace this path carves: a 129^3 grid with either
// precision (mixed: 47.2 MiB) fits, 257^3 does not.
constexpr size_t kScratchBytes = size_t(48) << 20;
constexpr int kScratchDevices = 16;

// One copy per device, held from the library's load until the process ends.
// Host code never uses this name as an address: each device's address comes
// from hipGetSymbolAddress below.
static __device__ __align__(256) char scratch[kScratchBytes];

struct ScratchSlot {
    std::mutex mu;        // one call at a time per device in this process
    char *dev = nullptr;  // this device's address of `scratch`
    mhs_plan plan;        // host bookkeeping of the hierarchy carved in it
    SolveState states[4]; // status read-back (pageable)
};
ScratchSlot g_scratch[kScratchDevices];
// descriptor staging, pageable: the call waits for its stream before it
// returns, so the next call may overwrite it
char g_scratch_stage[kScratchDevices][kStagingBytes];

} // namespace

extern "C" {

int mhs_solve_interior_noalloc(const mhs_grid *grid, const mhs_model *model, double *d_P, const mhs_opts *o,
                               mhs_info *info, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!grid || !d_P) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    int st = validate_opts(o);
    if (st) return st;
    size_t need = 0;
    if ((st = mhs_workspace_bytes(grid, o->precision, &need))) return st;
    if (need - kAlign > kScratchBytes)
        return fail(MHS_ERR_WORKSPACE, "grid %dx%dx%d needs %zu bytes of scratch, the library holds %zu", grid->nx,
                    grid->ny, grid->nz, need - kAlign, kScratchBytes);
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices)
        return fail(MHS_ERR_UNSUPPORTED, "device %d: the scratch path serves devices 0..%d", dev,
                    kScratchDevices - 1);
    ScratchSlot &slot = g_scratch[dev];
    std::lock_guard<std::mutex> lock(slot.mu);
    if (!slot.dev) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr % kAlign) != 0) return fail(MHS_ERR_HIP, "scratch symbol address is unusable");
        slot.dev = (char *)ptr;
    }
    mhs_plan &p = slot.plan;
    p = mhs_plan();
    p.precisions = o->precision;
    p.device = dev;
    p.graphs_ok = false; // a capture stream and graph objects would be allocations
    if ((st = geometry(&p, grid))) return st;
    if ((st = validate_model(&p, model, false))) return st;
    p.ws = slot.dev;
    p.ws_bytes = kScratchBytes;
    const size_t used = carve_plan(&p, p.ws, o->precision) - kAlign;
    p.stage.host = g_scratch_stage[dev];
    p.h_states = slot.states;
    hipStream_t s = (hipStream_t)stream;
    // the previous call's contents: coarse boundary nodes must read as zero
    HIPCHK(launch_zero(p.ws, (used + 15) & ~size_t(15), s));
    st = solve_interior_on(&p, model, d_P, o, info, s, t0);
    // nothing of this call may still run when the next one clears the array
    const hipError_t e = hipStreamSynchronize(s);
    if (st == MHS_OK && e != hipSuccess)
        return fail(MHS_ERR_HIP, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    return st;
}

} // extern "C"
