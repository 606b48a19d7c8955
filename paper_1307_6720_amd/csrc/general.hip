// The general scalar elliptic problem of Section 2.2,
//     a(x) lap u + b(x) u = c(x) in D,  u given on the boundary of D,
// in the interior of the box (3D Laplacian) or on one of its faces (2D), with
// per-node coefficients: FP64 V-cycles on the divided form
//     lap_h u + beta u = gamma,  beta = b/a,  gamma = c/a,
// which has the same discrete solution.
//
// Unlike the solve of (8), whose coefficients depend on z only and live in
// per-plane tables, every stage here reads per-node beta, so the kernels are
// one thread per node (or per node of one colour), reading neighbours
// through the caches: each level's arrays are streamed once or twice per
// stage and the coarse levels are small.  The hierarchy (shapes and which
// axes a step halves) is the one of (8), so the grid transfers are the same
// full weighting and linear interpolation, applied per axis.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "plan.h"

namespace mhs {

// Largest coarsest grid solved exactly (dense elimination in LDS).
constexpr int kGenMaxCoarse = 96;
constexpr int kGenThreads = 256;

// One level of a general problem as a kernel sees it.
struct GenItem {
    double *u;           // iterate (level 0: the solution array)
    double *f;           // right-hand side gamma (level 0: c / a)
    double *beta;        // b / a (sampled at this level's nodes)
    double *r;           // residual of this level (for the restriction)
    double *uc, *fc;     // next coarser level: iterate and right-hand side
    double *betac;       // next coarser level: beta (filled by the prep)
    const double *a, *b, *c; // level 0 prep: the caller's coefficients
    SolveState *state;   // stages are skipped once state->done != 0
    double *partials;    // per-block sums (norm) or {max beta, bad count} (prep)
    double cx, cy, cz;   // 1 / h^2 per axis (cz = 0 on a face)
    int32_t nx, ny, nz;  // nodes (nz = 1 on a face)
    int32_t ncx, ncy, ncz;
    int32_t sx, sz;      // fine nodes per coarse node along x and y (1|2), along z (1|2)
    int32_t planar, warm;
};

struct GenHier {
    Hierarchy geo;          // shapes, spacings, step kinds (keepz, keepxy)
    bool ok = false;        // geometry built
    double *u0 = nullptr;   // faces: level-0 iterate (a copy of the face)
    double *u[kMaxLevels] = {}, *f[kMaxLevels] = {}, *beta[kMaxLevels] = {}, *r[kMaxLevels] = {};
    double *partials = nullptr;
    int npart = 0;
};

struct GenPlan {
    GenHier h[4]; // 0: 3D, 1: (x, y) faces, 2: (y, z) faces, 3: (x, z) faces
};

void GenPlanDeleter::operator()(GenPlan *g) const { delete g; }

namespace {

__device__ __forceinline__ bool gen_skip(const GenItem &it) { return it.state && it.state->done; }

__device__ __forceinline__ double gen_block_sum(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kGenThreads / 64; ++q) s += red[q];
    return s;
}

// Interior node t (of mx * my * mz, x fastest) -> (i, j, k).
__device__ __forceinline__ void gen_node(int64_t t, const GenItem &it, int &i, int &j, int &k)
{
    const int mx = it.nx - 2, my = it.ny - 2;
    i = 1 + (int)(t % mx);
    const int64_t q = t / mx;
    j = 1 + (int)(q % my);
    k = it.planar ? 0 : 1 + (int)(q / my);
}

__device__ __forceinline__ int64_t gen_interior(const GenItem &it)
{
    return (int64_t)(it.nx - 2) * (it.ny - 2) * (it.planar ? 1 : it.nz - 2);
}

// Level 0: beta = b/a and gamma = c/a on interior nodes (0 elsewhere), the
// interior of u zeroed unless warm-started; per block the largest beta and
// the number of interior nodes whose a vanishes or whose a, b, c are not
// finite.
__global__ __launch_bounds__(kGenThreads) void k_gen_prep(const GenItem *__restrict__ itp)
{
    __shared__ double red[kGenThreads / 64];
    const GenItem &it = *itp;
    const int64_t N = (int64_t)it.nx * it.ny * it.nz;
    const int64_t e = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    double bmax = -INFINITY, bad = 0.0;
    if (e < N) {
        const int i = (int)(e % it.nx);
        const int64_t q = e / it.nx;
        const int j = (int)(q % it.ny), k = (int)(q / it.ny);
        const bool in = i >= 1 && i <= it.nx - 2 && j >= 1 && j <= it.ny - 2 &&
                        (it.planar ? k == 0 : (k >= 1 && k <= it.nz - 2));
        double be = 0.0, ge = 0.0;
        if (in) {
            const double av = it.a[e], bv = it.b[e], cv = it.c[e];
            if (!(av != 0.0 && isfinite(av) && isfinite(bv) && isfinite(cv))) bad = 1.0;
            be = bv / av;
            ge = cv / av;
            bmax = be;
            if (!it.warm) it.u[e] = 0.0;
        }
        it.beta[e] = be;
        it.f[e] = ge;
    }
    // block maximum and count (fixed order)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        bmax = fmax(bmax, __shfl_down(bmax, o, 64));
        bad += __shfl_down(bad, o, 64);
    }
    __shared__ double redb[kGenThreads / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w] = bmax;
        redb[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = -INFINITY, c = 0.0;
        for (int q = 0; q < kGenThreads / 64; ++q) {
            m = fmax(m, red[q]);
            c += redb[q];
        }
        it.partials[2 * blockIdx.x] = m;
        it.partials[2 * blockIdx.x + 1] = c;
    }
}

// Reduce the prep's per-block pairs into out[0] = max beta, out[1] = count.
__global__ __launch_bounds__(kGenThreads) void k_gen_prep_reduce(const double *__restrict__ partials, int n,
                                                                 double *out)
{
    __shared__ double red[kGenThreads], redb[kGenThreads];
    double m = -INFINITY, c = 0.0;
    for (int q = threadIdx.x; q < n; q += kGenThreads) {
        m = fmax(m, partials[2 * q]);
        c += partials[2 * q + 1];
    }
    red[threadIdx.x] = m;
    redb[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kGenThreads; ++q) {
            m = fmax(m, red[q]);
            c += redb[q];
        }
        out[0] = m;
        out[1] = c;
    }
}

// beta of the next coarser level: its value at the coincident fine node.
__global__ __launch_bounds__(kGenThreads) void k_gen_inject(const GenItem *__restrict__ itp)
{
    const GenItem &it = *itp;
    const int64_t N = (int64_t)it.ncx * it.ncy * it.ncz;
    const int64_t e = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    if (e >= N) return;
    const int I = (int)(e % it.ncx);
    const int64_t q = e / it.ncx;
    const int J = (int)(q % it.ncy), K = (int)(q / it.ncy);
    it.betac[e] = it.beta[(int64_t)(it.sx * I) + it.nx * ((int64_t)(it.sx * J) + (int64_t)it.ny * (it.sz * K))];
}

// One colour of a red-black Gauss-Seidel sweep: each interior node with
// (i + j + k) % 2 == colour solves its row of lap_h u + beta u = gamma for
// itself (its neighbours all have the other colour).  Thread t takes the
// colour's node among x-pair q of row (j, k).
__global__ __launch_bounds__(kGenThreads) void k_gen_sweep(const GenItem *__restrict__ itp, int colour)
{
    const GenItem &it = *itp;
    if (gen_skip(it)) return;
    const int mx = it.nx - 2, my = it.ny - 2;
    const int half = (mx + 1) >> 1;
    const int64_t t = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    const int q = (int)(t % half);
    const int64_t rest = t / half;
    const int j = 1 + (int)(rest % my);
    const int k = it.planar ? 0 : 1 + (int)(rest / my);
    if (it.planar ? rest >= my : k > it.nz - 2) return;
    const int i = 1 + 2 * q + ((colour + 1 + j + k) & 1);
    if (i > it.nx - 2) return;
    const int64_t sxy = (int64_t)it.nx * it.ny;
    const int64_t e = i + (int64_t)it.nx * j + sxy * k;
    const double *u = it.u;
    double off = it.cx * (u[e + 1] + u[e - 1]) + it.cy * (u[e + it.nx] + u[e - it.nx]);
    if (!it.planar) off += it.cz * (u[e + sxy] + u[e - sxy]);
    const double sum = 2.0 * (it.cx + it.cy + it.cz);
    it.u[e] = (it.f[e] - off) / (it.beta[e] - sum);
}

// r = gamma - (lap_h u + beta u) on interior nodes (boundary entries of r
// stay zero); with `norm`, per-block sums of r^2 for the stopping rule.
__global__ __launch_bounds__(kGenThreads) void k_gen_resid(const GenItem *__restrict__ itp, int norm)
{
    __shared__ double red[kGenThreads / 64];
    const GenItem &it = *itp;
    if (gen_skip(it)) return;
    const int64_t t = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    double rr = 0.0;
    if (t < gen_interior(it)) {
        int i, j, k;
        gen_node(t, it, i, j, k);
        const int64_t sxy = (int64_t)it.nx * it.ny;
        const int64_t e = i + (int64_t)it.nx * j + sxy * k;
        const double *u = it.u;
        double off = it.cx * (u[e + 1] + u[e - 1]) + it.cy * (u[e + it.nx] + u[e - it.nx]);
        if (!it.planar) off += it.cz * (u[e + sxy] + u[e - sxy]);
        const double sum = 2.0 * (it.cx + it.cy + it.cz);
        const double r = it.f[e] - (off + (it.beta[e] - sum) * u[e]);
        if (it.r) it.r[e] = r;
        rr = r * r;
    }
    if (norm) {
        const double s = gen_block_sum(rr, red);
        if (threadIdx.x == 0) it.partials[blockIdx.x] = s;
    }
}

// Full weighting of r onto the coarse interior nodes: weights 1/4, 1/2, 1/4
// along each halved axis, the coincident node along a kept one.
__global__ __launch_bounds__(kGenThreads) void k_gen_restrict(const GenItem *__restrict__ itp)
{
    const GenItem &it = *itp;
    if (gen_skip(it)) return;
    const int mcx = it.ncx - 2, mcy = it.ncy - 2, mcz = it.planar ? 1 : it.ncz - 2;
    const int64_t t = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    if (t >= (int64_t)mcx * mcy * mcz) return;
    const int I = 1 + (int)(t % mcx);
    const int64_t q = t / mcx;
    const int J = 1 + (int)(q % mcy);
    const int K = it.planar ? 0 : 1 + (int)(q / mcy);
    const double w[3] = {0.25, 0.5, 0.25};
    const int rx = it.sx == 2 ? 1 : 0, rz = it.sz == 2 ? 1 : 0;
    const int64_t sxy = (int64_t)it.nx * it.ny;
    double s = 0.0;
    for (int c = -rz; c <= rz; ++c)
        for (int b = -rx; b <= rx; ++b)
            for (int a = -rx; a <= rx; ++a) {
                const double wt = (rx ? w[a + 1] * w[b + 1] : 1.0) * (rz ? w[c + 1] : 1.0);
                const int64_t e = (it.sx * I + a) + (int64_t)it.nx * (it.sx * J + b) + sxy * (it.sz * K + c);
                s += wt * it.r[e];
            }
    it.fc[I + (int64_t)it.ncx * J + (int64_t)it.ncx * it.ncy * K] = s;
}

// u += I(u_c) on fine interior nodes: along a halved axis an even index
// takes the coincident coarse node, an odd one the mean of its two
// neighbours; along a kept axis the same index.
__global__ __launch_bounds__(kGenThreads) void k_gen_prolong(const GenItem *__restrict__ itp)
{
    const GenItem &it = *itp;
    if (gen_skip(it)) return;
    const int64_t t = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    if (t >= gen_interior(it)) return;
    int i, j, k;
    gen_node(t, it, i, j, k);
    const int64_t csxy = (int64_t)it.ncx * it.ncy;
    const int I0 = it.sx == 2 ? i >> 1 : i, I1 = it.sx == 2 ? (i + 1) >> 1 : i;
    const int J0 = it.sx == 2 ? j >> 1 : j, J1 = it.sx == 2 ? (j + 1) >> 1 : j;
    const int K0 = it.sz == 2 ? k >> 1 : k, K1 = it.sz == 2 ? (k + 1) >> 1 : k;
    double s = 0.0;
    for (int K = K0; K <= K1; ++K)
        for (int J = J0; J <= J1; ++J)
            for (int I = I0; I <= I1; ++I) {
                const double wx = (I0 == I1) ? 1.0 : 0.5, wy = (J0 == J1) ? 1.0 : 0.5, wz = (K0 == K1) ? 1.0 : 0.5;
                s += wx * wy * wz * it.uc[I + (int64_t)it.ncx * J + csxy * K];
            }
    it.u[i + (int64_t)it.nx * j + (int64_t)it.nx * it.ny * k] += s;
}

// Exact solve of the coarsest grid (zero boundary values): the dense
// operator of its m interior unknowns assembled in LDS, Gaussian elimination
// (the negated operator is positive definite, so no pivoting), then back
// substitution.  One workgroup.
__global__ __launch_bounds__(kGenThreads) void k_gen_coarsest(const GenItem *__restrict__ itp)
{
    const GenItem &it = *itp;
    if (gen_skip(it)) return;
    __shared__ double M[kGenMaxCoarse * kGenMaxCoarse];
    __shared__ double rhs[kGenMaxCoarse], lf[kGenMaxCoarse];
    const int mx = it.nx - 2, my = it.ny - 2, mz = it.planar ? 1 : it.nz - 2;
    const int m = mx * my * mz;
    const int k0 = it.planar ? 0 : 1;
    const int64_t sxy = (int64_t)it.nx * it.ny;
    const double sum = 2.0 * (it.cx + it.cy + it.cz);
    for (int e = threadIdx.x; e < m * m; e += kGenThreads) M[e] = 0.0;
    __syncthreads();
    for (int r = threadIdx.x; r < m; r += kGenThreads) {
        const int i = 1 + r % mx, j = 1 + (r / mx) % my, k = k0 + r / (mx * my);
        const int64_t e = i + (int64_t)it.nx * j + sxy * k;
        M[r * m + r] = it.beta[e] - sum;
        if (i > 1) M[r * m + r - 1] = it.cx;
        if (i < it.nx - 2) M[r * m + r + 1] = it.cx;
        if (j > 1) M[r * m + r - mx] = it.cy;
        if (j < it.ny - 2) M[r * m + r + mx] = it.cy;
        if (!it.planar && k > 1) M[r * m + r - mx * my] = it.cz;
        if (!it.planar && k < it.nz - 2) M[r * m + r + mx * my] = it.cz;
        rhs[r] = it.f[e];
    }
    __syncthreads();
    for (int p = 0; p < m; ++p) {
        for (int r = p + 1 + threadIdx.x; r < m; r += kGenThreads) lf[r] = M[r * m + p] / M[p * m + p];
        __syncthreads();
        const int w = m - p; // columns p .. m-1
        for (int e = threadIdx.x; e < (m - p - 1) * w; e += kGenThreads) {
            const int r = p + 1 + e / w, c = p + e % w;
            M[r * m + c] -= lf[r] * M[p * m + c];
        }
        for (int r = p + 1 + threadIdx.x; r < m; r += kGenThreads) rhs[r] -= lf[r] * rhs[p];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int r = m - 1; r >= 0; --r) {
            double s = rhs[r];
            for (int c = r + 1; c < m; ++c) s -= M[r * m + c] * rhs[c];
            rhs[r] = s / M[r * m + r];
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < m; r += kGenThreads) {
        const int i = 1 + r % mx, j = 1 + (r / mx) % my, k = k0 + r / (mx * my);
        it.u[i + (int64_t)it.nx * j + sxy * k] = rhs[r];
    }
}

// Face of the box <-> a contiguous (n2, n1) array: gather (to_face = 0)
// copies the whole face, scatter (to_face = 1) writes back its interior.
struct FaceMap {
    double *P;
    double *v;
    int32_t nx, ny, nz;
    int32_t face, n1, n2, to_face;
};

__global__ __launch_bounds__(kGenThreads) void k_gen_face(FaceMap fm)
{
    const int64_t t = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    if (t >= (int64_t)fm.n1 * fm.n2) return;
    const int a = (int)(t % fm.n1), b = (int)(t / fm.n1);
    if (fm.to_face && (a == 0 || a == fm.n1 - 1 || b == 0 || b == fm.n2 - 1)) return;
    int i = 0, j = 0, k = 0;
    switch (fm.face) {
    case MHS_FACE_BASE: i = a; j = b; k = 0; break;
    case MHS_FACE_TOP: i = a; j = b; k = fm.nz - 1; break;
    case MHS_FACE_XLO: i = 0; j = a; k = b; break;
    case MHS_FACE_XHI: i = fm.nx - 1; j = a; k = b; break;
    case MHS_FACE_YLO: i = a; j = 0; k = b; break;
    default: i = a; j = fm.ny - 1; k = b; break;
    }
    const int64_t e = i + (int64_t)fm.nx * (j + (int64_t)fm.ny * k);
    if (fm.to_face)
        fm.P[e] = fm.v[t];
    else
        fm.v[t] = fm.P[e];
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kGenThreads - 1) / kGenThreads); }

} // namespace

hipError_t gen_exec(const Launch &L, hipStream_t s)
{
    const GenItem *it = (const GenItem *)L.items;
    const unsigned nb = blocks_for(L.n);
    switch (L.kind) {
    case Launch::kGenSweep:
        hipLaunchKernelGGL(k_gen_sweep, dim3(nb), dim3(kGenThreads), 0, s, it, L.flags);
        break;
    case Launch::kGenResid:
        hipLaunchKernelGGL(k_gen_resid, dim3(nb), dim3(kGenThreads), 0, s, it, L.flags);
        break;
    case Launch::kGenRestrict:
        hipLaunchKernelGGL(k_gen_restrict, dim3(nb), dim3(kGenThreads), 0, s, it);
        break;
    case Launch::kGenProlong:
        hipLaunchKernelGGL(k_gen_prolong, dim3(nb), dim3(kGenThreads), 0, s, it);
        break;
    case Launch::kGenCoarsest:
        hipLaunchKernelGGL(k_gen_coarsest, dim3(1), dim3(kGenThreads), 0, s, it);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- host side ----------------------------------------------------------------

namespace {

int64_t interior_count(const Level &lv, bool planar)
{
    return (int64_t)(lv.n[0] - 2) * (lv.n[1] - 2) * (planar ? 1 : lv.n[2] - 2);
}

void carve_gen(GenHier &g, Carver &cv, bool face)
{
    const Hierarchy &h = g.geo;
    if (face) g.u0 = cv.take<double>(h.lv[0].N);
    for (int l = 0; l < h.L; ++l) {
        const size_t N = h.lv[l].N;
        if (l > 0) g.u[l] = cv.take<double>(N);
        g.f[l] = cv.take<double>(N);
        g.beta[l] = cv.take<double>(N);
        if (l + 1 < h.L) g.r[l] = cv.take<double>(N);
    }
    g.npart = (int)std::max<int64_t>(blocks_for((int64_t)h.lv[0].N), blocks_for(interior_count(h.lv[0], h.planar)));
    g.partials = cv.take<double>(2 * (size_t)g.npart + 2);
}

// Smallest eigenvalue of -lap_h (zero boundary) on a level.
double lap_lambda_min(const Level &lv, bool planar)
{
    const double pi = 3.14159265358979323846;
    double s = 0.0;
    for (int a = 0; a < (planar ? 2 : 3); ++a) {
        const double t = std::sin(pi / (2.0 * (lv.n[a] - 1)));
        s += 4.0 / (lv.h[a] * lv.h[a]) * t * t;
    }
    return s;
}

GenItem level_item(const GenHier &g, int l, double *u, SolveState *state)
{
    const Hierarchy &h = g.geo;
    const Level &lv = h.lv[l];
    GenItem it{};
    it.u = u;
    it.f = g.f[l];
    it.beta = g.beta[l];
    it.r = g.r[l];
    it.state = state;
    it.partials = g.partials;
    it.cx = 1.0 / (lv.h[0] * lv.h[0]);
    it.cy = 1.0 / (lv.h[1] * lv.h[1]);
    it.cz = h.planar ? 0.0 : 1.0 / (lv.h[2] * lv.h[2]);
    it.nx = lv.n[0];
    it.ny = lv.n[1];
    it.nz = lv.n[2];
    it.planar = h.planar ? 1 : 0;
    if (l + 1 < h.L) {
        const Level &c = h.lv[l + 1];
        it.uc = g.u[l + 1];
        it.fc = g.f[l + 1];
        it.betac = g.beta[l + 1];
        it.ncx = c.n[0];
        it.ncy = c.n[1];
        it.ncz = c.n[2];
        it.sx = lv.keepxy ? 1 : 2;
        it.sz = (h.planar || lv.keepz) ? 1 : 2;
    }
    return it;
}

Launch gen_launch(Launch::Kind kind, const GenItem *d, int64_t threads, int flags, double bytes)
{
    Launch L{};
    L.kind = kind;
    L.items = d;
    L.n = threads;
    L.flags = flags;
    L.prof = MHS_PROF_GENERAL;
    L.bytes = bytes;
    return L;
}

// One V(nu1, nu2) cycle from level l down, appended to pg.
void add_gen_vcycle(Program &pg, const GenHier &g, const GenItem *const *items, int l, int nu1, int nu2)
{
    const Hierarchy &h = g.geo;
    const Level &lv = h.lv[l];
    const int64_t in = interior_count(lv, h.planar);
    const int64_t half = (int64_t)((lv.n[0] - 1) / 2) * (lv.n[1] - 2) * (h.planar ? 1 : lv.n[2] - 2);
    // algorithmic bytes: a sweep reads u, beta, gamma and writes u once (half
    // per colour launch); the residual reads u, beta, gamma and writes r
    const double N = (double)lv.N;
    if (l == h.L - 1) {
        pg.launches.push_back(gen_launch(Launch::kGenCoarsest, items[l], 1, 0, 24.0 * N));
        return;
    }
    if (l > 0) {
        Launch z{};
        z.kind = Launch::kZero;
        z.dst = g.u[l];
        z.n = (int64_t)((lv.N * sizeof(double) + 15) & ~size_t(15));
        pg.launches.push_back(z);
    }
    for (int s = 0; s < nu1; ++s)
        for (int c = 0; c < 2; ++c) pg.launches.push_back(gen_launch(Launch::kGenSweep, items[l], half, c, 16.0 * N));
    pg.launches.push_back(gen_launch(Launch::kGenResid, items[l], in, 0, 32.0 * N));
    const Level &cl = h.lv[l + 1];
    pg.launches.push_back(gen_launch(Launch::kGenRestrict, items[l], interior_count(cl, h.planar), 0,
                                     8.0 * (N + (double)cl.N)));
    add_gen_vcycle(pg, g, items, l + 1, nu1, nu2);
    pg.launches.push_back(gen_launch(Launch::kGenProlong, items[l], in, 0, 16.0 * N + 8.0 * (double)cl.N));
    for (int s = 0; s < nu2; ++s)
        for (int c = 0; c < 2; ++c) pg.launches.push_back(gen_launch(Launch::kGenSweep, items[l], half, c, 16.0 * N));
}

// Solve on hierarchy g with level-0 iterate u0 (boundary values = data).
int gen_solve(mhs_plan *p, GenHier &g, double *u0, const double *a, const double *b, const double *c,
              const mhs_opts *o, mhs_info *info, hipStream_t s, std::chrono::steady_clock::time_point t0)
{
    const Hierarchy &h = g.geo;
    const int L = h.L;
    if (h.m > kGenMaxCoarse)
        return fail(MHS_ERR_UNSUPPORTED, "the coarsest grid has %d unknowns (the general solve takes at most %d)", h.m,
                    kGenMaxCoarse);
    int st = begin_staging(p);
    if (st) return st;
    SolveState *d_state = (SolveState *)p->stage.put(initial_state(o->rtol, o->max_cycles));
    const GenItem *items[kMaxLevels] = {};
    for (int l = 0; l < L; ++l) {
        GenItem it = level_item(g, l, l == 0 ? u0 : g.u[l], d_state);
        if (l == 0) {
            it.a = a;
            it.b = b;
            it.c = c;
            it.warm = o->warm_start;
        }
        items[l] = p->stage.put(it);
    }
    // the prep item writes its per-block pairs to partials; the reduction
    // result goes after them
    double *d_red = g.partials + 2 * (size_t)g.npart;
    Program cyc;
    {
        Launch chk = gen_launch(Launch::kGenResid, items[0], interior_count(h.lv[0], h.planar), 1,
                                24.0 * (double)h.lv[0].N);
        chk.pre = true;
        cyc.launches.push_back(chk);
        add_finalize(cyc, p->stage, g.partials, (int)blocks_for(interior_count(h.lv[0], h.planar)), d_state);
        cyc.launches.back().pre = true;
        add_gen_vcycle(cyc, g, items, 0, o->nu1, o->nu2);
    }
    if (!d_state || !items[L - 1] || !cyc.ok) return fail(MHS_ERR_WORKSPACE, "staging area exhausted");
    if ((st = flush_staging(p, s))) return st;
    // level-0 coefficients, then beta on every coarser level
    const int64_t N0 = (int64_t)h.lv[0].N;
    hipLaunchKernelGGL(k_gen_prep, dim3(blocks_for(N0)), dim3(kGenThreads), 0, s, items[0]);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_gen_prep_reduce, dim3(1), dim3(kGenThreads), 0, s, g.partials, (int)blocks_for(N0), d_red);
    HIPCHK(hipGetLastError());
    for (int l = 0; l + 1 < L; ++l) {
        hipLaunchKernelGGL(k_gen_inject, dim3(blocks_for((int64_t)h.lv[l + 1].N)), dim3(kGenThreads), 0, s, items[l]);
        HIPCHK(hipGetLastError());
    }
    // definiteness and the coefficients' validity, read back once
    double hred[2] = {0.0, 0.0};
    HIPCHK(hipMemcpyAsync(p->h_states, d_red, sizeof hred, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(hred, p->h_states, sizeof hred);
    if (hred[1] != 0.0)
        return fail(MHS_ERR_INVALID_ARG, "a vanishes, or a, b or c is not finite, at %.0f interior nodes", hred[1]);
    const double lam = lap_lambda_min(h.lv[L - 1], h.planar);
    if (!(hred[0] < 0.5 * lam))
        return fail(MHS_ERR_INDEFINITE, "max b/a = %g is not below half the smallest eigenvalue of -lap on the "
                    "coarsest grid (%g)", hred[0], 0.5 * lam);
    SolveState fin{};
    int syncs = 1;
    if ((st = drive(p, cyc, d_state, o, &fin, &syncs, s, kSolveGeneral))) return st;
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
        return fail(status, "general solve stopped after %d cycles (relative residual %g)", fin.checks - 1,
                    fin.r0 > 0 ? fin.rnorm / fin.r0 : 0.0);
    return MHS_OK;
}

int gen_check(mhs_plan *p, const mhs_opts *o)
{
    if (!p) return fail(MHS_ERR_INVALID_ARG, "NULL plan");
    int st = validate_opts(o);
    if (st) return st;
    if (!p->gen) return fail(MHS_ERR_UNSUPPORTED, "plan was created without MHS_PLAN_GENERAL");
    if (o->precision != MHS_PREC_FP64) return fail(MHS_ERR_UNSUPPORTED, "the general solve runs in FP64 only");
    return set_device(p);
}

} // namespace

void gen_create(mhs_plan *p, Carver &cv)
{
    if (!p->gen) {
        p->gen.reset(new GenPlan());
        const mhs_grid &gr = p->grid;
        const int n3[3] = {gr.nx, gr.ny, gr.nz};
        const double l3[3] = {gr.lx, gr.ly, gr.lz};
        GenHier *H = p->gen->h;
        H[0].ok = build_geometry(H[0].geo, n3, l3, false) == MHS_OK;
        const int nf[3][3] = {{gr.nx, gr.ny, 1}, {gr.ny, gr.nz, 1}, {gr.nx, gr.nz, 1}};
        const double lf[3][3] = {{gr.lx, gr.ly, 1.0}, {gr.ly, gr.lz, 1.0}, {gr.lx, gr.lz, 1.0}};
        for (int q = 0; q < 3; ++q) H[q + 1].ok = build_geometry(H[q + 1].geo, nf[q], lf[q], true) == MHS_OK;
        fail(MHS_OK, "%s", ""); // geometry messages of unusable hierarchies are reported at solve time
    }
    for (int q = 0; q < 4; ++q)
        if (p->gen->h[q].ok) carve_gen(p->gen->h[q], cv, q > 0);
}

} // namespace mhs

using namespace mhs;

extern "C" {

int mhs_solve_general(mhs_plan *p, const double *d_a, const double *d_b, const double *d_c, double *d_u,
                      const mhs_opts *o, mhs_info *info, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    int st = gen_check(p, o);
    if (st) return st;
    if (!d_a || !d_b || !d_c || !d_u) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    GenHier &g = p->gen->h[0];
    if (!g.ok) return fail(MHS_ERR_UNSUPPORTED, "grid has no multigrid hierarchy for the general operator");
    return gen_solve(p, g, d_u, d_a, d_b, d_c, o, info, (hipStream_t)stream, t0);
}

int mhs_solve_face(mhs_plan *p, int32_t face, const double *d_a, const double *d_b, const double *d_c, double *d_P,
                   const mhs_opts *o, mhs_info *info, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    int st = gen_check(p, o);
    if (st) return st;
    if (!d_a || !d_b || !d_c || !d_P) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    if (face < MHS_FACE_BASE || face > MHS_FACE_YHI) return fail(MHS_ERR_INVALID_ARG, "face must be 0..5");
    const int which = face <= MHS_FACE_TOP ? 1 : (face <= MHS_FACE_XHI ? 2 : 3);
    GenHier &g = p->gen->h[which];
    if (!g.ok) return fail(MHS_ERR_UNSUPPORTED, "face grid has no multigrid hierarchy");
    hipStream_t s = (hipStream_t)stream;
    FaceMap fm{d_P, g.u0, p->grid.nx, p->grid.ny, p->grid.nz, face, g.geo.lv[0].n[0], g.geo.lv[0].n[1], 0};
    const int64_t nf = (int64_t)fm.n1 * fm.n2;
    hipLaunchKernelGGL(k_gen_face, dim3(blocks_for(nf)), dim3(kGenThreads), 0, s, fm);
    HIPCHK(hipGetLastError());
    st = gen_solve(p, g, g.u0, d_a, d_b, d_c, o, info, s, t0);
    if (st != MHS_OK && st != MHS_ERR_NO_CONVERGENCE && st != MHS_ERR_DIVERGED) return st;
    // the iterate goes back to the face in every case (as the other solves
    // leave their last iterate in place)
    fm.to_face = 1;
    hipLaunchKernelGGL(k_gen_face, dim3(blocks_for(nf)), dim3(kGenThreads), 0, s, fm);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return st;
}

} // extern "C"
