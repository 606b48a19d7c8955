// gfx950 kernels of the multigrid path for the NR99 linear MHS potential.
//
// The discrete operator at an interior node of level l (equation (8) of
// Section 2.2 with central differences; the 2D operator of (11) is the
// same with cz = 0 and xi = 0):
//   (A u) = cx_k (uE + uW) + cy_k (uN + uS) + cz (uU + uD) + d_k u,
//   cx_k = (1 - xi_k)/dx^2, cy_k = (1 - xi_k)/dy^2, cz = 1/dz^2,
//   d_k = alpha^2 - 2 cx_k - 2 cy_k - 2 cz.
// Arrays are x-fastest: idx = i + nx (j + ny k).
//
// All stencil kernels are HBM-bound (a few flops per 8-16 bytes), so they
// are built around coalesced x-rows, LDS tiles with recomputed halos and
// z-marching, not around matrix cores.
#include "internal.h"

namespace mhs {
namespace {

template <typename Item>
__device__ __forceinline__ int find_item(const Item *items, int n, int tile)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile_base <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fixed-order block sum (deterministic); result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) s += red[q];
    }
    return s;
}

// Trilinear interpolation of the coarse correction at fine node (i, j, k):
// coincident nodes copy, edge/face/cell midpoints average 2/4/8 values.
template <typename T>
__device__ __forceinline__ T interp3(const T *__restrict__ ec, int ncx, int ncy, int i, int j, int k)
{
    const size_t sy = (size_t)ncx, sz = (size_t)ncx * ncy;
    const T *p = ec + (size_t)(i >> 1) + sy * (size_t)(j >> 1) + sz * (size_t)(k >> 1);
    const int oi = i & 1, oj = j & 1, ok = k & 1;
    const T h = (T)0.5;
    auto X = [&](const T *q) { return oi ? h * (q[0] + q[1]) : q[0]; };
    auto Y = [&](const T *q) { return oj ? h * (X(q) + X(q + sy)) : X(q); };
    return ok ? h * (Y(p) + Y(p + sz)) : Y(p);
}

template <typename T>
__device__ __forceinline__ T interp2(const T *__restrict__ ec, int ncx, int i, int j)
{
    const size_t sy = (size_t)ncx;
    const T *p = ec + (size_t)(i >> 1) + sy * (size_t)(j >> 1);
    const int oi = i & 1, oj = j & 1;
    const T h = (T)0.5;
    auto X = [&](const T *q) { return oi ? h * (q[0] + q[1]) : q[0]; };
    return oj ? h * (X(p) + X(p + sy)) : X(p);
}

// ============================================================================
// 3D red-black Gauss-Seidel sweep, ping-pong (u_in -> u_out).
//
// A workgroup owns kTX x kTY interior nodes of kKZ consecutive planes.  It
// stages a (kTY+4) x (kTX+4) window of each plane in LDS (four planes in
// flight) and marches up in z: at step s it updates the red nodes of plane
// s on the tile plus a one-node ring, then the black nodes of plane s-1 on
// the tile, whose red neighbours (planes s-2, s-1, s) are all final by
// then.  Red nodes of the ring are recomputed from u_in, so neighbouring
// tiles never read each other's output and one pass is one complete sweep,
// identical to updating all red nodes and then all black nodes.
// ============================================================================
constexpr int kWX = kTX + 4;
constexpr int kWY = kTY + 4;
constexpr int kRedPerRow = kTX / 2 + 1;
constexpr int kBlackPerRow = kTX / 2;
constexpr int kOwn = kTY * kTX / kThreads;
static_assert(kTY * kTX % kThreads == 0, "tile must be a multiple of the block");

template <typename T, int FLAGS>
__global__ __launch_bounds__(kThreads) void k_sweep3(const LevelItem *__restrict__ items, int nitems)
{
    constexpr bool HAS_F = (FLAGS & kHasF) != 0;
    constexpr bool ZERO_IN = (FLAGS & kZeroIn) != 0;
    constexpr bool NORM = (FLAGS & kNorm) != 0;
    constexpr bool PROLONG = (FLAGS & kProlong) != 0;
    __shared__ T S[4][kWY][kWX];
    __shared__ double red[kThreads / 64];

    const int tile = blockIdx.x;
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && it->state->done) return;
    const T *__restrict__ uin = (const T *)it->u_in;
    T *__restrict__ uout = (T *)it->u_out;
    const T *__restrict__ f = (const T *)it->f;
    const T *__restrict__ ec = (const T *)it->ec;
    const T *__restrict__ coef = (const T *)it->coef;
    const T cz = (T)it->cz;
    const int nx = it->nx, ny = it->ny, nz = it->nz;
    const int ncx = it->ncx, ncy = it->ncy;
    int local = tile - it->tile_base;
    const int tx = local % it->ntx;
    local /= it->ntx;
    const int ty = local % it->nty;
    const int tz = local / it->nty;
    const int i0 = 1 + tx * kTX, j0 = 1 + ty * kTY;
    const int kb = 1 + tz * kKZ;
    const int ke = min(kb + kKZ, nz - 1);
    const size_t sxy = (size_t)nx * ny;
    const int tid = threadIdx.x;

    auto load_plane = [&](int p) {
        T(*dst)[kWX] = S[p & 3];
        for (int e = tid; e < kWY * kWX; e += kThreads) {
            const int w = e / kWX, c = e - w * kWX;
            const int i = i0 - 2 + c, j = j0 - 2 + w;
            T v = (T)0;
            if (i >= 0 && i < nx && j >= 0 && j < ny) {
                const size_t idx = (size_t)i + (size_t)nx * j + sxy * p;
                if constexpr (!ZERO_IN) v = uin[idx];
                if constexpr (PROLONG) {
                    if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && p >= 1 && p <= nz - 2)
                        v += interp3(ec, ncx, ncy, i, j, p);
                }
            }
            dst[w][c] = v;
        }
    };

    double acc = 0.0;
    T below[kOwn];
#pragma unroll
    for (int q = 0; q < kOwn; ++q) below[q] = (T)0;

    if (kb - 2 >= 0) load_plane(kb - 2);
    load_plane(kb - 1);
    for (int s = kb - 1; s <= ke; ++s) {
        if (s + 1 <= nz - 1) load_plane(s + 1);
        __syncthreads();
        if constexpr (NORM) {
            // residual of the input iterate at plane s (all values still old);
            // the old plane s-1 comes from registers captured one step earlier
            T(*P)[kWX] = S[s & 3];
            T(*Pp)[kWX] = S[(s + 1) & 3];
            const bool do_res = (s >= kb && s < ke);
            T cx = 0, cy = 0, d = 0;
            if (do_res) {
                cx = coef[4 * s];
                cy = coef[4 * s + 1];
                d = coef[4 * s + 2];
            }
#pragma unroll
            for (int q = 0; q < kOwn; ++q) {
                const int e = tid + q * kThreads;
                const int w = 2 + e / kTX, c = 2 + e % kTX;
                const T uc = P[w][c];
                if (do_res) {
                    const int i = i0 + c - 2, j = j0 + w - 2;
                    if (i <= nx - 2 && j <= ny - 2) {
                        T fv = (T)0;
                        if constexpr (HAS_F) fv = f[(size_t)i + (size_t)nx * j + sxy * s];
                        const T r = fv - (cx * (P[w][c + 1] + P[w][c - 1]) + cy * (P[w + 1][c] + P[w - 1][c]) +
                                          cz * (Pp[w][c] + below[q]) + d * uc);
                        acc += (double)r * (double)r;
                    }
                }
                below[q] = uc;
            }
            __syncthreads();
        }
        // red nodes of plane s on the tile and its one-node ring
        if (s >= 1 && s <= nz - 2) {
            const T cx = coef[4 * s], cy = coef[4 * s + 1], invd = coef[4 * s + 3];
            T(*P)[kWX] = S[s & 3];
            T(*Pm)[kWX] = S[(s - 1) & 3];
            T(*Pp)[kWX] = S[(s + 1) & 3];
            for (int e = tid; e < (kTY + 2) * kRedPerRow; e += kThreads) {
                const int w = 1 + e / kRedPerRow;
                const int q = e - (w - 1) * kRedPerRow;
                const int c = 1 + ((i0 + j0 + w + s + 1) & 1) + 2 * q;
                const int i = i0 - 2 + c, j = j0 - 2 + w;
                if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) {
                    T fv = (T)0;
                    if constexpr (HAS_F) fv = f[(size_t)i + (size_t)nx * j + sxy * s];
                    P[w][c] = (fv - (cx * (P[w][c + 1] + P[w][c - 1]) + cy * (P[w + 1][c] + P[w - 1][c]) +
                                     cz * (Pp[w][c] + Pm[w][c]))) *
                              invd;
                }
            }
        }
        __syncthreads();
        // black nodes of plane m = s - 1 on the tile
        const int m = s - 1;
        if (m >= kb && m < ke) {
            const T cx = coef[4 * m], cy = coef[4 * m + 1], invd = coef[4 * m + 3];
            T(*P)[kWX] = S[m & 3];
            T(*Pm)[kWX] = S[(m - 1) & 3];
            T(*Pp)[kWX] = S[(m + 1) & 3];
            for (int e = tid; e < kTY * kBlackPerRow; e += kThreads) {
                const int w = 2 + e / kBlackPerRow;
                const int q = e - (w - 2) * kBlackPerRow;
                const int c = 2 + ((i0 + j0 + w + m + 1) & 1) + 2 * q;
                const int i = i0 - 2 + c, j = j0 - 2 + w;
                if (i <= nx - 2 && j <= ny - 2) {
                    T fv = (T)0;
                    if constexpr (HAS_F) fv = f[(size_t)i + (size_t)nx * j + sxy * m];
                    P[w][c] = (fv - (cx * (P[w][c + 1] + P[w][c - 1]) + cy * (P[w + 1][c] + P[w - 1][c]) +
                                     cz * (Pp[w][c] + Pm[w][c]))) *
                              invd;
                }
            }
        }
        __syncthreads();
        if (m >= kb && m < ke) {
            T(*P)[kWX] = S[m & 3];
            for (int e = tid; e < kTY * kTX; e += kThreads) {
                const int w = 2 + e / kTX, c = 2 + e % kTX;
                const int i = i0 + c - 2, j = j0 + w - 2;
                if (i <= nx - 2 && j <= ny - 2) uout[(size_t)i + (size_t)nx * j + sxy * m] = P[w][c];
            }
        }
    }
    if constexpr (NORM) {
        const double tot = block_sum<kThreads>(acc, red);
        if (tid == 0) it->partials[tile - it->tile_base] = tot;
    }
}

// ============================================================================
// 2D red-black sweep for equation (11): one plane, ping-pong.
// ============================================================================
constexpr int kW2X = kTX + 4;
constexpr int kW2Y = kTY2 + 4;
constexpr int kOwn2 = kTY2 * kTX / kThreads;
static_assert(kTY2 * kTX % kThreads == 0, "tile must be a multiple of the block");

template <typename T, int FLAGS>
__global__ __launch_bounds__(kThreads) void k_sweep2(const LevelItem *__restrict__ items, int nitems)
{
    constexpr bool HAS_F = (FLAGS & kHasF) != 0;
    constexpr bool ZERO_IN = (FLAGS & kZeroIn) != 0;
    constexpr bool NORM = (FLAGS & kNorm) != 0;
    constexpr bool PROLONG = (FLAGS & kProlong) != 0;
    __shared__ T S[kW2Y][kW2X];
    __shared__ double red[kThreads / 64];

    const int tile = blockIdx.x;
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && it->state->done) return;
    const T *__restrict__ uin = (const T *)it->u_in;
    T *__restrict__ uout = (T *)it->u_out;
    const T *__restrict__ f = (const T *)it->f;
    const T *__restrict__ ec = (const T *)it->ec;
    const T *__restrict__ coef = (const T *)it->coef;
    const int nx = it->nx, ny = it->ny;
    const int ncx = it->ncx;
    const int local = tile - it->tile_base;
    const int tx = local % it->ntx, ty = local / it->ntx;
    const int i0 = 1 + tx * kTX, j0 = 1 + ty * kTY2;
    const int tid = threadIdx.x;
    const T cx = coef[0], cy = coef[1], d = coef[2], invd = coef[3];

    for (int e = tid; e < kW2Y * kW2X; e += kThreads) {
        const int w = e / kW2X, c = e - w * kW2X;
        const int i = i0 - 2 + c, j = j0 - 2 + w;
        T v = (T)0;
        if (i >= 0 && i < nx && j >= 0 && j < ny) {
            if constexpr (!ZERO_IN) v = uin[(size_t)i + (size_t)nx * j];
            if constexpr (PROLONG) {
                if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) v += interp2(ec, ncx, i, j);
            }
        }
        S[w][c] = v;
    }
    __syncthreads();
    double acc = 0.0;
    if constexpr (NORM) {
#pragma unroll
        for (int q = 0; q < kOwn2; ++q) {
            const int e = tid + q * kThreads;
            const int w = 2 + e / kTX, c = 2 + e % kTX;
            const int i = i0 + c - 2, j = j0 + w - 2;
            if (i <= nx - 2 && j <= ny - 2) {
                T fv = (T)0;
                if constexpr (HAS_F) fv = f[(size_t)i + (size_t)nx * j];
                const T r = fv - (cx * (S[w][c + 1] + S[w][c - 1]) + cy * (S[w + 1][c] + S[w - 1][c]) + d * S[w][c]);
                acc += (double)r * (double)r;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < (kTY2 + 2) * kRedPerRow; e += kThreads) {
        const int w = 1 + e / kRedPerRow;
        const int q = e - (w - 1) * kRedPerRow;
        const int c = 1 + ((i0 + j0 + w + 1) & 1) + 2 * q;
        const int i = i0 - 2 + c, j = j0 - 2 + w;
        if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) {
            T fv = (T)0;
            if constexpr (HAS_F) fv = f[(size_t)i + (size_t)nx * j];
            S[w][c] = (fv - (cx * (S[w][c + 1] + S[w][c - 1]) + cy * (S[w + 1][c] + S[w - 1][c]))) * invd;
        }
    }
    __syncthreads();
    for (int e = tid; e < kTY2 * kBlackPerRow; e += kThreads) {
        const int w = 2 + e / kBlackPerRow;
        const int q = e - (w - 2) * kBlackPerRow;
        const int c = 2 + ((i0 + j0 + w + 1) & 1) + 2 * q;
        const int i = i0 - 2 + c, j = j0 - 2 + w;
        if (i <= nx - 2 && j <= ny - 2) {
            T fv = (T)0;
            if constexpr (HAS_F) fv = f[(size_t)i + (size_t)nx * j];
            S[w][c] = (fv - (cx * (S[w][c + 1] + S[w][c - 1]) + cy * (S[w + 1][c] + S[w - 1][c]))) * invd;
        }
    }
    __syncthreads();
    for (int e = tid; e < kTY2 * kTX; e += kThreads) {
        const int w = 2 + e / kTX, c = 2 + e % kTX;
        const int i = i0 + c - 2, j = j0 + w - 2;
        if (i <= nx - 2 && j <= ny - 2) uout[(size_t)i + (size_t)nx * j] = S[w][c];
    }
    if constexpr (NORM) {
        const double tot = block_sum<kThreads>(acc, red);
        if (tid == 0) it->partials[tile - it->tile_base] = tot;
    }
}

// ============================================================================
// 3D residual r = f - A u (on the fly) + full weighting onto coarse nodes:
//   f_c(I,J,K) = sum_{a,b,c in -1..1} w_a w_b w_c r(2I+a, 2J+b, 2K+c),
//   w_0 = 1/2, w_{+-1} = 1/4.
// A workgroup owns kCX x kCY coarse nodes and marches kKC coarse planes; each
// fine plane's residual is computed once into LDS from an LDS-staged window
// of u (three planes in flight) and folded into the coarse sums.
// ============================================================================
constexpr int kRWX = 2 * kCX + 3;
constexpr int kRWY = 2 * kCY + 3;
constexpr int kRRX = 2 * kCX + 1;
constexpr int kRRY = 2 * kCY + 1;
static_assert(kCX * kCY == kThreads, "one coarse node per thread");

template <typename T, bool HAS_F>
__global__ __launch_bounds__(kThreads) void k_restrict3(const LevelItem *__restrict__ items, int nitems)
{
    __shared__ T U[3][kRWY][kRWX];
    __shared__ T R[kRRY][kRRX];

    const int tile = blockIdx.x;
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && it->state->done) return;
    const T *__restrict__ u = (const T *)it->u_in;
    const T *__restrict__ f = (const T *)it->f;
    T *__restrict__ fc = (T *)it->u_out;
    const T *__restrict__ coef = (const T *)it->coef;
    const T cz = (T)it->cz;
    const int nx = it->nx, ny = it->ny, nz = it->nz;
    const int ncx = it->ncx, ncy = it->ncy, ncz = it->ncz;
    int local = tile - it->tile_base;
    const int tx = local % it->ntx;
    local /= it->ntx;
    const int ty = local % it->nty;
    const int tz = local / it->nty;
    const int I0 = 1 + tx * kCX, J0 = 1 + ty * kCY;
    const int Kb = 1 + tz * kKC;
    const int Ke = min(Kb + kKC, ncz - 1);
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1; // residual window origin
    const int ui0 = fi0 - 1, uj0 = fj0 - 1;       // u window origin
    const size_t sxy = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const int tI = tid % kCX, tJ = tid / kCX;
    const int I = I0 + tI, J = J0 + tJ;
    const bool valid = (I <= ncx - 2) && (J <= ncy - 2);

    auto load_u = [&](int p) {
        T(*dst)[kRWX] = U[p % 3];
        for (int e = tid; e < kRWY * kRWX; e += kThreads) {
            const int w = e / kRWX, c = e - w * kRWX;
            const int i = ui0 + c, j = uj0 + w;
            T v = (T)0;
            if (i >= 0 && i < nx && j >= 0 && j < ny) v = u[(size_t)i + (size_t)nx * j + sxy * p];
            dst[w][c] = v;
        }
    };

    load_u(2 * Kb - 2);
    load_u(2 * Kb - 1);
    T acc = (T)0;
    const T q4 = (T)0.25, h2 = (T)0.5;
    for (int m = 2 * Kb - 1; m <= 2 * Ke - 1; ++m) {
        load_u(m + 1);
        __syncthreads();
        {
            const T cx = coef[4 * m], cy = coef[4 * m + 1], d = coef[4 * m + 2];
            T(*P)[kRWX] = U[m % 3];
            T(*Pm)[kRWX] = U[(m + 2) % 3];
            T(*Pp)[kRWX] = U[(m + 1) % 3];
            for (int e = tid; e < kRRY * kRRX; e += kThreads) {
                const int w = e / kRRX, c = e - w * kRRX;
                const int i = fi0 + c, j = fj0 + w;
                T r = (T)0;
                if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) {
                    const int uw = w + 1, uc = c + 1;
                    T fv = (T)0;
                    if constexpr (HAS_F) fv = f[(size_t)i + (size_t)nx * j + sxy * m];
                    r = fv - (cx * (P[uw][uc + 1] + P[uw][uc - 1]) + cy * (P[uw + 1][uc] + P[uw - 1][uc]) +
                              cz * (Pp[uw][uc] + Pm[uw][uc]) + d * P[uw][uc]);
                }
                R[w][c] = r;
            }
        }
        __syncthreads();
        const int cw = 2 * tJ + 1, cc = 2 * tI + 1;
        auto row = [&](int w) { return q4 * R[w][cc - 1] + h2 * R[w][cc] + q4 * R[w][cc + 1]; };
        const T s2 = q4 * row(cw - 1) + h2 * row(cw) + q4 * row(cw + 1);
        if (m & 1) {
            const int Kend = (m - 1) >> 1;
            if (Kend >= Kb) {
                acc += q4 * s2;
                if (valid) fc[(size_t)I + (size_t)ncx * J + (size_t)ncx * ncy * Kend] = acc;
            }
            acc = q4 * s2;
        } else {
            acc += h2 * s2;
        }
        __syncthreads();
    }
    (void)nz;
}

// 2D residual + nine-point full weighting.  One coarse node per thread,
// residual computed into LDS for the fine window.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict2(const LevelItem *__restrict__ items, int nitems)
{
    __shared__ T U[kRWY][kRWX];
    __shared__ T R[kRRY][kRRX];
    const int tile = blockIdx.x;
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && it->state->done) return;
    const T *__restrict__ u = (const T *)it->u_in;
    const T *__restrict__ f = (const T *)it->f;
    T *__restrict__ fc = (T *)it->u_out;
    const T *__restrict__ coef = (const T *)it->coef;
    const int nx = it->nx, ny = it->ny;
    const int ncx = it->ncx, ncy = it->ncy;
    const int local = tile - it->tile_base;
    const int tx = local % it->ntx, ty = local / it->ntx;
    const int I0 = 1 + tx * kCX, J0 = 1 + ty * kCY;
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1;
    const int ui0 = fi0 - 1, uj0 = fj0 - 1;
    const int tid = threadIdx.x;
    const int tI = tid % kCX, tJ = tid / kCX;
    const int I = I0 + tI, J = J0 + tJ;
    const T cx = coef[0], cy = coef[1], d = coef[2];
    for (int e = tid; e < kRWY * kRWX; e += kThreads) {
        const int w = e / kRWX, c = e - w * kRWX;
        const int i = ui0 + c, j = uj0 + w;
        U[w][c] = (i >= 0 && i < nx && j >= 0 && j < ny) ? u[(size_t)i + (size_t)nx * j] : (T)0;
    }
    __syncthreads();
    for (int e = tid; e < kRRY * kRRX; e += kThreads) {
        const int w = e / kRRX, c = e - w * kRRX;
        const int i = fi0 + c, j = fj0 + w;
        T r = (T)0;
        if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) {
            const int uw = w + 1, uc = c + 1;
            r = f[(size_t)i + (size_t)nx * j] -
                (cx * (U[uw][uc + 1] + U[uw][uc - 1]) + cy * (U[uw + 1][uc] + U[uw - 1][uc]) + d * U[uw][uc]);
        }
        R[w][c] = r;
    }
    __syncthreads();
    if (I <= ncx - 2 && J <= ncy - 2) {
        const T q4 = (T)0.25, h2 = (T)0.5;
        const int cw = 2 * tJ + 1, cc = 2 * tI + 1;
        auto row = [&](int w) { return q4 * R[w][cc - 1] + h2 * R[w][cc] + q4 * R[w][cc + 1]; };
        fc[(size_t)I + (size_t)ncx * J] = q4 * row(cw - 1) + h2 * row(cw) + q4 * row(cw + 1);
    }
}

// ============================================================================
// Iterative refinement, FP64 part: u_out = u_in + e (e from the FP32 inner
// solve, zero on boundaries) and r = -A u_out at level 0 (the right-hand side
// of (8) is zero; the data enter through the Dirichlet plane k = 0), written
// as FP32 for the next inner solve, plus per-tile FP64 sums of r^2.
// ============================================================================
constexpr int kIWX = kTX + 2;
constexpr int kIWY = kTY + 2;

template <bool HAS_E>
__global__ __launch_bounds__(kThreads) void k_ir3(const LevelItem *__restrict__ items, int nitems)
{
    __shared__ double S[3][kIWY][kIWX];
    __shared__ double red[kThreads / 64];
    const int tile = blockIdx.x;
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && it->state->done) return;
    const double *__restrict__ uin = (const double *)it->u_in;
    double *__restrict__ uout = (double *)it->u_out;
    const float *__restrict__ e32 = (const float *)it->ec;
    float *__restrict__ r32 = (float *)it->r_out;
    const double *__restrict__ coef = (const double *)it->coef;
    const double cz = it->cz;
    const int nx = it->nx, ny = it->ny, nz = it->nz;
    int local = tile - it->tile_base;
    const int tx = local % it->ntx;
    local /= it->ntx;
    const int ty = local % it->nty;
    const int tz = local / it->nty;
    const int i0 = 1 + tx * kTX, j0 = 1 + ty * kTY;
    const int kb = 1 + tz * kKZ;
    const int ke = min(kb + kKZ, nz - 1);
    const size_t sxy = (size_t)nx * ny;
    const int tid = threadIdx.x;

    auto load_plane = [&](int p) {
        double(*dst)[kIWX] = S[p % 3];
        for (int e = tid; e < kIWY * kIWX; e += kThreads) {
            const int w = e / kIWX, c = e - w * kIWX;
            const int i = i0 - 1 + c, j = j0 - 1 + w;
            double v = 0.0;
            if (i >= 0 && i < nx && j >= 0 && j < ny) {
                const size_t idx = (size_t)i + (size_t)nx * j + sxy * p;
                v = uin[idx];
                if constexpr (HAS_E) {
                    if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && p >= 1 && p <= nz - 2)
                        v += (double)e32[idx];
                }
            }
            dst[w][c] = v;
        }
    };
    double acc = 0.0;
    load_plane(kb - 1);
    load_plane(kb);
    for (int m = kb; m < ke; ++m) {
        load_plane(m + 1);
        __syncthreads();
        const double cx = coef[4 * m], cy = coef[4 * m + 1], d = coef[4 * m + 2];
        double(*P)[kIWX] = S[m % 3];
        double(*Pm)[kIWX] = S[(m + 2) % 3];
        double(*Pp)[kIWX] = S[(m + 1) % 3];
        for (int e = tid; e < kTY * kTX; e += kThreads) {
            const int w = 1 + e / kTX, c = 1 + e % kTX;
            const int i = i0 + c - 1, j = j0 + w - 1;
            if (i <= nx - 2 && j <= ny - 2) {
                const size_t idx = (size_t)i + (size_t)nx * j + sxy * m;
                const double uc = P[w][c];
                const double r = -(cx * (P[w][c + 1] + P[w][c - 1]) + cy * (P[w + 1][c] + P[w - 1][c]) +
                                   cz * (Pp[w][c] + Pm[w][c]) + d * uc);
                if constexpr (HAS_E) uout[idx] = uc;
                r32[idx] = (float)r;
                acc += r * r;
            }
        }
        __syncthreads();
    }
    const double tot = block_sum<kThreads>(acc, red);
    if (tid == 0) it->partials[tile - it->tile_base] = tot;
}

// ============================================================================
// Bottom solver: one workgroup runs a whole V(nu1,nu2) cycle over the small
// levels of one request, from a zero initial guess, in FP64, with exact
// red-black Gauss-Seidel ordering (barrier between colours) and an exact
// dense solve on the coarsest grid.  Work arrays live in the workspace and
// stay cache resident.
// ============================================================================
__device__ __forceinline__ void bottom_smooth(const BottomItem &b, int l, int nsweeps)
{
    const int nx = b.n[l][0], ny = b.n[l][1], nz = b.n[l][2];
    const bool planar = b.planar != 0;
    const int mx = nx - 2, my = ny - 2, mz = planar ? 1 : nz - 2;
    const int nint = mx * my * mz;
    double *__restrict__ u = b.u[l];
    const double *__restrict__ f = b.f[l];
    const double *__restrict__ coef = b.coef[l];
    const double cz = b.cz[l];
    const size_t sxy = (size_t)nx * ny;
    for (int s = 0; s < nsweeps; ++s) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int e = threadIdx.x; e < nint; e += kBottomThreads) {
                const int ii = e % mx, rest = e / mx;
                const int jj = rest % my, kk = rest / my;
                const int i = ii + 1, j = jj + 1, k = planar ? 0 : kk + 1;
                if (((i + j + k) & 1) != colour) continue;
                const size_t idx = (size_t)i + (size_t)nx * j + sxy * k;
                const int kc = planar ? 0 : k;
                const double cx = coef[4 * kc], cy = coef[4 * kc + 1], invd = coef[4 * kc + 3];
                double off = cx * (u[idx + 1] + u[idx - 1]) + cy * (u[idx + nx] + u[idx - nx]);
                if (!planar) off += cz * (u[idx + sxy] + u[idx - sxy]);
                u[idx] = (f[idx] - off) * invd;
            }
            __syncthreads();
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBottomThreads) void k_bottom(const BottomItem *__restrict__ items, int nitems)
{
    const BottomItem &b = items[blockIdx.x];
    if (b.state && b.state->done) return;
    const bool planar = b.planar != 0;
    const int tid = threadIdx.x;
    {
        const size_t N0 = (size_t)b.n[0][0] * b.n[0][1] * b.n[0][2];
        const T *ft = (const T *)b.f_top;
        for (size_t e = tid; e < N0; e += kBottomThreads) {
            b.f[0][e] = (double)ft[e];
            b.u[0][e] = 0.0;
        }
    }
    __syncthreads();
    const int L = b.nlev;
    for (int l = 0; l < L - 1; ++l) {
        const int nx = b.n[l][0], ny = b.n[l][1], nz = b.n[l][2];
        const size_t sxy = (size_t)nx * ny;
        if (l > 0) {
            const size_t N = sxy * nz;
            for (size_t e = tid; e < N; e += kBottomThreads) b.u[l][e] = 0.0;
            __syncthreads();
        }
        bottom_smooth(b, l, b.nu1);
        // residual on interior nodes
        {
            const int mx = nx - 2, my = ny - 2, mz = planar ? 1 : nz - 2;
            const int nint = mx * my * mz;
            const double *__restrict__ u = b.u[l];
            const double *__restrict__ f = b.f[l];
            const double *__restrict__ coef = b.coef[l];
            const double cz = b.cz[l];
            for (int e = tid; e < nint; e += kBottomThreads) {
                const int ii = e % mx, rest = e / mx;
                const int jj = rest % my, kk = rest / my;
                const int i = ii + 1, j = jj + 1, k = planar ? 0 : kk + 1;
                const size_t idx = (size_t)i + (size_t)nx * j + sxy * k;
                const int kc = planar ? 0 : k;
                double au = coef[4 * kc] * (u[idx + 1] + u[idx - 1]) + coef[4 * kc + 1] * (u[idx + nx] + u[idx - nx]) +
                            coef[4 * kc + 2] * u[idx];
                if (!planar) au += cz * (u[idx + sxy] + u[idx - sxy]);
                b.r[idx] = f[idx] - au;
            }
        }
        __syncthreads();
        // full weighting onto the interior of level l+1
        {
            const int cnx = b.n[l + 1][0], cny = b.n[l + 1][1], cnz = b.n[l + 1][2];
            const int mx = cnx - 2, my = cny - 2, mz = planar ? 1 : cnz - 2;
            const int nint = mx * my * mz;
            const double *__restrict__ r = b.r;
            double *__restrict__ fc = b.f[l + 1];
            for (int e = tid; e < nint; e += kBottomThreads) {
                const int ii = e % mx, rest = e / mx;
                const int jj = rest % my, kk = rest / my;
                const int I = ii + 1, J = jj + 1, K = planar ? 0 : kk + 1;
                const size_t fidx = (size_t)(2 * I) + (size_t)nx * (2 * J) + sxy * (planar ? 0 : 2 * K);
                auto row = [&](size_t q) { return 0.25 * r[q - 1] + 0.5 * r[q] + 0.25 * r[q + 1]; };
                auto pl = [&](size_t q) { return 0.25 * row(q - nx) + 0.5 * row(q) + 0.25 * row(q + nx); };
                double v = planar ? pl(fidx) : 0.25 * pl(fidx - sxy) + 0.5 * pl(fidx) + 0.25 * pl(fidx + sxy);
                fc[(size_t)I + (size_t)cnx * J + (size_t)cnx * cny * K] = v;
            }
        }
        __syncthreads();
    }
    // exact solve on the coarsest grid: u = Minv f over interior nodes
    {
        const int nx = b.n[L - 1][0], ny = b.n[L - 1][1], nz = b.n[L - 1][2];
        const int mx = nx - 2, my = ny - 2;
        const size_t sxy = (size_t)nx * ny;
        const int m = b.m;
        double *__restrict__ u = b.u[L - 1];
        const double *__restrict__ f = b.f[L - 1];
        if (L > 1) {
            const size_t N = sxy * nz;
            for (size_t e = tid; e < N; e += kBottomThreads) u[e] = 0.0;
        }
        __syncthreads();
        for (int p = tid; p < m; p += kBottomThreads) {
            double s = 0.0;
            for (int q = 0; q < m; ++q) {
                const int qi = q % mx, qr = q / mx;
                const int qj = qr % my, qk = qr / my;
                const size_t fidx = (size_t)(qi + 1) + (size_t)nx * (qj + 1) + sxy * (planar ? 0 : qk + 1);
                s += b.minv[(size_t)p * m + q] * f[fidx];
            }
            const int pi = p % mx, pr = p / mx;
            const int pj = pr % my, pk = pr / my;
            u[(size_t)(pi + 1) + (size_t)nx * (pj + 1) + sxy * (planar ? 0 : pk + 1)] = s;
        }
        __syncthreads();
    }
    for (int l = L - 2; l >= 0; --l) {
        const int nx = b.n[l][0], ny = b.n[l][1], nz = b.n[l][2];
        const int cnx = b.n[l + 1][0], cny = b.n[l + 1][1];
        const size_t sxy = (size_t)nx * ny;
        const int mx = nx - 2, my = ny - 2, mz = planar ? 1 : nz - 2;
        const int nint = mx * my * mz;
        double *__restrict__ u = b.u[l];
        const double *__restrict__ ec = b.u[l + 1];
        for (int e = tid; e < nint; e += kBottomThreads) {
            const int ii = e % mx, rest = e / mx;
            const int jj = rest % my, kk = rest / my;
            const int i = ii + 1, j = jj + 1, k = planar ? 0 : kk + 1;
            const double v = planar ? interp2(ec, cnx, i, j) : interp3(ec, cnx, cny, i, j, k);
            u[(size_t)i + (size_t)nx * j + sxy * k] += v;
        }
        __syncthreads();
        bottom_smooth(b, l, b.nu2);
    }
    {
        const size_t N0 = (size_t)b.n[0][0] * b.n[0][1] * b.n[0][2];
        T *ut = (T *)b.u_top;
        for (size_t e = tid; e < N0; e += kBottomThreads) ut[e] = (T)b.u[0][e];
    }
}

// ============================================================================
// Convergence check: fixed-order sum of the per-tile partials, then the
// stopping rule ||r_c|| <= rtol ||r_0|| (or divergence, or the cap).
// ============================================================================
__global__ __launch_bounds__(kThreads) void k_finalize(const FinalizeItem *__restrict__ items, int nitems)
{
    __shared__ double red[kThreads / 64];
    const FinalizeItem &it = items[blockIdx.x];
    SolveState *st = it.state;
    if (st->done) return;
    double s = 0.0;
    for (int i = threadIdx.x; i < it.n; i += kThreads) s += it.partials[i];
    s = block_sum<kThreads>(s, red);
    if (threadIdx.x == 0) {
        const double rn = sqrt(s);
        const int c = st->checks;
        if (c == 0) st->r0 = rn;
        const double r0 = st->r0;
        int32_t done = kRunning;
        if (!(rn <= 1.0e300))
            done = kDiverged; // NaN or Inf
        else if (rn <= st->rtol * r0)
            done = kConverged;
        else if (rn > 10.0 * r0)
            done = kDiverged;
        else if (c >= st->max_iter)
            done = kMaxed;
        st->rnorm = rn;
        st->checks = c + 1;
        st->done = done;
    }
}

// ============================================================================
// Field recovery (Section 2.2): B by central differences of P, p and rho from
// (9) and (10).  A workgroup owns kTX x kFY nodes of kKZ planes; P planes are
// staged in LDS with a two-node halo and Bz planes with a one-node halo,
// three planes of each in flight.  Side and top faces: B = 0.  Base plane:
// one-sided second-order z-derivatives.
// ============================================================================
constexpr int kFPX = kTX + 4;
constexpr int kFPY = kFY + 4;
constexpr int kFBX = kTX + 2;
constexpr int kFBY = kFY + 2;

__global__ __launch_bounds__(kThreads) void k_fields(const FieldsItem *__restrict__ items, int nitems)
{
    __shared__ double SP[3][kFPY][kFPX];
    __shared__ double SB[3][kFBY][kFBX];
    const int tile = blockIdx.x;
    const FieldsItem *it = items + find_item(items, nitems, tile);
    const double *__restrict__ P = it->P;
    const int nx = it->nx, ny = it->ny, nz = it->nz;
    int local = tile - it->tile_base;
    const int tx = local % it->ntx;
    local /= it->ntx;
    const int ty = local % it->nty;
    const int tz = local / it->nty;
    const int i0 = tx * kTX, j0 = ty * kFY;
    const int kb = tz * kKZ;
    const int ke = min(kb + kKZ, nz);
    const size_t sxy = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const double ix2 = 1.0 / (it->dx * it->dx), iy2 = 1.0 / (it->dy * it->dy);
    const double i2dx = 0.5 / it->dx, i2dy = 0.5 / it->dy, i2dz = 0.5 / it->dz;
    const double alpha = it->alpha, mu0 = it->mu0, g = it->g;
    const double *tab = it->tab;

    auto load_plane = [&](int p) {
        double(*dst)[kFPX] = SP[p % 3];
        for (int e = tid; e < kFPY * kFPX; e += kThreads) {
            const int w = e / kFPX, c = e - w * kFPX;
            const int i = i0 - 2 + c, j = j0 - 2 + w;
            dst[w][c] = (i >= 0 && i < nx && j >= 0 && j < ny) ? P[(size_t)i + (size_t)nx * j + sxy * p] : 0.0;
        }
    };
    auto bz_plane = [&](int p) {
        double(*src)[kFPX] = SP[p % 3];
        double(*dst)[kFBX] = SB[p % 3];
        for (int e = tid; e < kFBY * kFBX; e += kThreads) {
            const int w = e / kFBX, c = e - w * kFBX;
            const int i = i0 - 1 + c, j = j0 - 1 + w;
            double v = 0.0;
            if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && p <= nz - 2) {
                const int pw = w + 1, pc = c + 1;
                v = -((src[pw][pc + 1] - 2.0 * src[pw][pc] + src[pw][pc - 1]) * ix2 +
                      (src[pw + 1][pc] - 2.0 * src[pw][pc] + src[pw - 1][pc]) * iy2);
            }
            dst[w][c] = v;
        }
    };

    int loaded = (kb == 0) ? -1 : kb - 2;
    for (int m = kb; m < ke; ++m) {
        if (m < nz - 1) {
            const int hi = min((m == 0) ? 2 : m + 1, nz - 1);
            while (loaded < hi) {
                ++loaded;
                load_plane(loaded);
                __syncthreads();
                bz_plane(loaded);
                __syncthreads();
            }
        }
        const double xi = tab[m], dxi = tab[nz + m], pb = tab[2 * nz + m], rhob = tab[3 * nz + m];
        for (int e = tid; e < kFY * kTX; e += kThreads) {
            const int w = e / kTX, c = e % kTX;
            const int i = i0 + c, j = j0 + w;
            if (i >= nx || j >= ny) continue;
            const size_t idx = (size_t)i + (size_t)nx * j + sxy * m;
            double bx = 0.0, by = 0.0, bz = 0.0, p = pb, rho = rhob;
            if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && m <= nz - 2) {
                const int pw = w + 2, pc = c + 2, bw = w + 1, bc = c + 1;
                double(*Pc)[kFPX] = SP[m % 3];
                double(*Bc)[kFBX] = SB[m % 3];
                double dzp_xp, dzp_xm, dzp_yp, dzp_ym, dbzz;
                if (m >= 1) {
                    double(*Pu)[kFPX] = SP[(m + 1) % 3];
                    double(*Pd)[kFPX] = SP[(m + 2) % 3];
                    dzp_xp = (Pu[pw][pc + 1] - Pd[pw][pc + 1]) * i2dz;
                    dzp_xm = (Pu[pw][pc - 1] - Pd[pw][pc - 1]) * i2dz;
                    dzp_yp = (Pu[pw + 1][pc] - Pd[pw + 1][pc]) * i2dz;
                    dzp_ym = (Pu[pw - 1][pc] - Pd[pw - 1][pc]) * i2dz;
                    dbzz = (SB[(m + 1) % 3][bw][bc] - SB[(m + 2) % 3][bw][bc]) * i2dz;
                } else {
                    double(*P1)[kFPX] = SP[1];
                    double(*P2)[kFPX] = SP[2];
                    auto one = [&](int a, int b) { return (-3.0 * Pc[a][b] + 4.0 * P1[a][b] - P2[a][b]) * i2dz; };
                    dzp_xp = one(pw, pc + 1);
                    dzp_xm = one(pw, pc - 1);
                    dzp_yp = one(pw + 1, pc);
                    dzp_ym = one(pw - 1, pc);
                    dbzz = (-3.0 * SB[0][bw][bc] + 4.0 * SB[1][bw][bc] - SB[2][bw][bc]) * i2dz;
                }
                bx = alpha * (Pc[pw + 1][pc] - Pc[pw - 1][pc]) * i2dy + (dzp_xp - dzp_xm) * i2dx;
                by = -alpha * (Pc[pw][pc + 1] - Pc[pw][pc - 1]) * i2dx + (dzp_yp - dzp_ym) * i2dy;
                bz = Bc[bw][bc];
                const double dbzx = (Bc[bw][bc + 1] - Bc[bw][bc - 1]) * i2dx;
                const double dbzy = (Bc[bw + 1][bc] - Bc[bw - 1][bc]) * i2dy;
                const double bz2 = bz * bz;
                p = pb - xi * bz2 / (2.0 * mu0);
                rho = rhob + (dxi * bz2 / (2.0 * mu0) + xi * (bx * dbzx + by * dbzy + bz * dbzz) / mu0) / g;
            }
            it->Bx[idx] = bx;
            it->By[idx] = by;
            it->Bz[idx] = bz;
            it->p[idx] = p;
            it->rho[idx] = rho;
        }
        __syncthreads();
    }
}

// ============================================================================
// Preparation and copies.
// ============================================================================
template <typename Item>
__device__ __forceinline__ int find_prep(const Item *items, int n, int64_t g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].base <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Interior start of (8): P = 0 on side and top faces and on the base edges,
// P = 0 in the interior (step 1 of the procedure) unless warm-started, and
// the twin's faces equal P's faces.
__global__ __launch_bounds__(256) void k_prep3(const PrepItem *__restrict__ items, int nitems)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const PrepItem &it = items[find_prep(items, nitems, g)];
    const int64_t e = g - it.base;
    if (e >= it.n) return;
    const int nx = it.nx, ny = it.ny, nz = it.nz;
    const int i = (int)(e % nx);
    const int64_t r = e / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    const bool side = (i == 0 || i == nx - 1 || j == 0 || j == ny - 1);
    if (k == 0) {
        if (side) it.P[e] = 0.0;
        if (it.twin) it.twin[e] = side ? 0.0 : it.P[e];
    } else if (side || k == nz - 1) {
        it.P[e] = 0.0;
        if (it.twin) it.twin[e] = 0.0;
    } else if (!it.warm) {
        it.P[e] = 0.0;
    }
}

// Start of (11): f = -Bz0 on interior nodes, P0 = 0 on the edges (and in
// the interior unless warm-started), twin edges 0.
__global__ __launch_bounds__(256) void k_prep2(const PrepItem *__restrict__ items, int nitems)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const PrepItem &it = items[find_prep(items, nitems, g)];
    const int64_t e = g - it.base;
    if (e >= it.n) return;
    const int nx = it.nx, ny = it.ny;
    const int i = (int)(e % nx), j = (int)(e / nx);
    const bool edge = (i == 0 || i == nx - 1 || j == 0 || j == ny - 1);
    it.f2[e] = edge ? 0.0 : -it.bz0[e];
    if (edge || !it.warm) it.P[e] = 0.0;
    if (edge && it.twin) it.twin[e] = 0.0;
}

// dst = src; skipped once `skip` (if given) reports a finished solve.
__global__ __launch_bounds__(256) void k_copy(const double *__restrict__ src, double *__restrict__ dst, int64_t n,
                                              const SolveState *skip)
{
    if (skip && skip->done) return;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = src[e];
}

template <typename T>
hipError_t sweep3_dispatch(const LevelItem *items, int nitems, int ntiles, int flags, hipStream_t s)
{
    dim3 grid(ntiles), block(kThreads);
    switch (flags & 15) {
#define MHS_CASE(F)                                                                      \
    case F:                                                                              \
        hipLaunchKernelGGL((k_sweep3<T, F>), grid, block, 0, s, items, nitems);         \
        break;
        MHS_CASE(0) MHS_CASE(1) MHS_CASE(2) MHS_CASE(3) MHS_CASE(4) MHS_CASE(5) MHS_CASE(6) MHS_CASE(7)
        MHS_CASE(8) MHS_CASE(9) MHS_CASE(12) MHS_CASE(13)
#undef MHS_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t sweep2_dispatch(const LevelItem *items, int nitems, int ntiles, int flags, hipStream_t s)
{
    dim3 grid(ntiles), block(kThreads);
    switch (flags & 15) {
#define MHS_CASE(F)                                                                      \
    case F:                                                                              \
        hipLaunchKernelGGL((k_sweep2<T, F>), grid, block, 0, s, items, nitems);         \
        break;
        MHS_CASE(0) MHS_CASE(1) MHS_CASE(2) MHS_CASE(3) MHS_CASE(4) MHS_CASE(5) MHS_CASE(6) MHS_CASE(7)
        MHS_CASE(8) MHS_CASE(9) MHS_CASE(12) MHS_CASE(13)
#undef MHS_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace

hipError_t launch_sweep3(const LevelItem *items, int nitems, int ntiles, int flags, bool dbl, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    return dbl ? sweep3_dispatch<double>(items, nitems, ntiles, flags, s)
               : sweep3_dispatch<float>(items, nitems, ntiles, flags, s);
}

hipError_t launch_sweep2(const LevelItem *items, int nitems, int ntiles, int flags, bool dbl, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    return dbl ? sweep2_dispatch<double>(items, nitems, ntiles, flags, s)
               : sweep2_dispatch<float>(items, nitems, ntiles, flags, s);
}

hipError_t launch_restrict3(const LevelItem *items, int nitems, int ntiles, bool has_f, bool dbl, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(kThreads);
    if (dbl) {
        if (has_f)
            hipLaunchKernelGGL((k_restrict3<double, true>), grid, block, 0, s, items, nitems);
        else
            hipLaunchKernelGGL((k_restrict3<double, false>), grid, block, 0, s, items, nitems);
    } else {
        if (has_f)
            hipLaunchKernelGGL((k_restrict3<float, true>), grid, block, 0, s, items, nitems);
        else
            hipLaunchKernelGGL((k_restrict3<float, false>), grid, block, 0, s, items, nitems);
    }
    return hipGetLastError();
}

hipError_t launch_restrict2(const LevelItem *items, int nitems, int ntiles, bool dbl, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(kThreads);
    if (dbl)
        hipLaunchKernelGGL((k_restrict2<double>), grid, block, 0, s, items, nitems);
    else
        hipLaunchKernelGGL((k_restrict2<float>), grid, block, 0, s, items, nitems);
    return hipGetLastError();
}

hipError_t launch_ir3(const LevelItem *items, int nitems, int ntiles, bool has_e, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(kThreads);
    if (has_e)
        hipLaunchKernelGGL((k_ir3<true>), grid, block, 0, s, items, nitems);
    else
        hipLaunchKernelGGL((k_ir3<false>), grid, block, 0, s, items, nitems);
    return hipGetLastError();
}

hipError_t launch_bottom(const BottomItem *items, int nitems, bool dbl, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    dim3 grid(nitems), block(kBottomThreads);
    if (dbl)
        hipLaunchKernelGGL((k_bottom<double>), grid, block, 0, s, items, nitems);
    else
        hipLaunchKernelGGL((k_bottom<float>), grid, block, 0, s, items, nitems);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeItem *items, int nitems, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(nitems), dim3(kThreads), 0, s, items, nitems);
    return hipGetLastError();
}

hipError_t launch_fields(const FieldsItem *items, int nitems, int ntiles, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fields, dim3(ntiles), dim3(kThreads), 0, s, items, nitems);
    return hipGetLastError();
}

hipError_t launch_prep3(const PrepItem *items, int nitems, int64_t nthreads, hipStream_t s)
{
    if (nthreads <= 0) return hipSuccess;
    const int64_t blocks = (nthreads + 255) / 256;
    hipLaunchKernelGGL(k_prep3, dim3((unsigned)blocks), dim3(256), 0, s, items, nitems);
    return hipGetLastError();
}

hipError_t launch_prep2(const PrepItem *items, int nitems, int64_t nthreads, hipStream_t s)
{
    if (nthreads <= 0) return hipSuccess;
    const int64_t blocks = (nthreads + 255) / 256;
    hipLaunchKernelGGL(k_prep2, dim3((unsigned)blocks), dim3(256), 0, s, items, nitems);
    return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, int64_t n, const SolveState *skip, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, skip);
    return hipGetLastError();
}

} // namespace mhs
