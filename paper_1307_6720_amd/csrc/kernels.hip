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

// Descriptor pointers arrive without an address space, which would make every
// access a FLAT instruction; FLAT counts against the LDS wait counter too, so
// each LDS barrier would also wait for all outstanding HBM loads.  All
// buffers are device (global) memory: say so.
#define MHS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const MHS_GLOBAL T *gin(const void *p)
{
    return (const MHS_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ MHS_GLOBAL T *gout(void *p)
{
    return (MHS_GLOBAL T *)p;
}
// Small read-only tables indexed by workgroup-uniform values (per-plane
// coefficients): the constant address space lets them use scalar loads,
// which do not share the vector-memory wait counter with the plane prefetch.
#define MHS_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const MHS_CONST T *gconst(const void *p)
{
    return (const MHS_CONST T *)p;
}

// One plane of an array as a buffer resource (base address and byte length
// in scalar registers): loads and stores then take a 32-bit per-lane byte
// offset with no 64-bit address arithmetic per access, and an offset at or
// past the length reads zero.  Word 3 selects raw 32-bit dword access.
constexpr int kBufWord3 = 0x00020000;
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const MHS_GLOBAL T *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, kBufWord3);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

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

// Workgroup barrier that orders LDS traffic only.  The kernels share data
// between threads exclusively through LDS, so the barrier must not wait for
// outstanding global loads (a plain __syncthreads() would, which drains the
// prefetch ring at every step) or stores.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8), each with its own L2.  Remap so that each XCD receives one
// contiguous range of tiles: neighbouring tiles, which re-read each other's
// halo rows, then share an L2 and run at about the same time.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile()
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int x = b % kXcds, q = b / kXcds;
    const int per = nb / kXcds, rem = nb % kXcds;
    return x * per + min(x, rem) + q;
}
// A launch whose items have different shapes (requests of several sizes
// merged by the batch) takes its tiles in dispatch order instead: its items'
// tiles march different numbers of planes, and contiguous ranges would give
// some XCDs only the long marches.
__device__ __forceinline__ int launch_tile(const LevelItem *items, int nitems)
{
    return (nitems > 1 && items[0].spread) ? (int)blockIdx.x : xcd_tile();
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
    lds_barrier();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) s += red[q];
    }
    return s;
}

// Trilinear interpolation of the coarse correction at fine node (i, j, k):
// coincident nodes copy, edge/face/cell midpoints average 2/4/8 values.
template <typename T, typename Ptr>
__device__ __forceinline__ T interp3(Ptr ec, int ncx, int ncy, int i, int j, int k)
{
    const size_t sy = (size_t)ncx, sz = (size_t)ncx * ncy;
    const Ptr p = ec + (size_t)(i >> 1) + sy * (size_t)(j >> 1) + sz * (size_t)(k >> 1);
    const int oi = i & 1, oj = j & 1, ok = k & 1;
    const T h = (T)0.5;
    auto X = [&](Ptr q) -> T { return oi ? h * (q[0] + q[1]) : (T)q[0]; };
    auto Y = [&](Ptr q) -> T { return oj ? h * (X(q) + X(q + sy)) : X(q); };
    return ok ? h * (Y(p) + Y(p + sz)) : Y(p);
}

template <typename T, typename Ptr>
__device__ __forceinline__ T interp2(Ptr ec, int ncx, int i, int j)
{
    const size_t sy = (size_t)ncx;
    const Ptr p = ec + (size_t)(i >> 1) + sy * (size_t)(j >> 1);
    const int oi = i & 1, oj = j & 1;
    const T h = (T)0.5;
    auto X = [&](Ptr q) -> T { return oi ? h * (q[0] + q[1]) : (T)q[0]; };
    return oj ? h * (X(p) + X(p + sy)) : X(p);
}

// ============================================================================
// 3D red-black Gauss-Seidel sweep, ping-pong (u_in -> u_out).
//
// A workgroup owns kTX x kSTY interior nodes of `kz` consecutive planes.  It
// stages a (kSTY+4) x (kTX+4) window of each plane of u in LDS (five slots)
// and marches up in z: at step s it updates the red nodes of plane
// s on the tile plus a one-node ring, then the black nodes of plane s-1 on
// the tile, whose red neighbours (planes s-2, s-1, s) are all final by
// then.  Red nodes of the ring are recomputed from u_in, so neighbouring
// tiles never read each other's output and one pass is one complete sweep,
// identical to updating all red nodes and then all black nodes.
//
// The right-hand side is needed only at the nodes a thread updates (two
// red, one black, and its own two for the residual), so it goes from memory
// straight into registers at those nodes, with no LDS staging.
//
// Loads run kDepth planes ahead of the stencil in a ring of register sets,
// so kDepth planes of HBM traffic are in flight per workgroup.  Every index
// a thread uses (staging cells, red and black nodes, written nodes) is fixed
// for the whole z-march and computed once.  With the prolongation-fused
// variant each register set also carries the coarse planes of the next fine
// plane; they are staged in LDS one step early and interpolated in z and y
// during the red phase, so staging a plane only adds the x interpolation.
// ============================================================================
constexpr int kWX = kTX + 4;
constexpr int kWY = kSTY + 4;
constexpr int kWCells = kWX * kWY;
// LDS rows store even columns first, then odd columns, so the colour phases
// (which touch every other column) read consecutive doubles: no bank conflicts
constexpr int kHalf = kWX / 2;
__device__ __forceinline__ int sx(int c) { return (c & 1) * kHalf + (c >> 1); }
static_assert(kWX % 2 == 0, "window width must be even");
constexpr int kWPer = (kWCells + kSThreads - 1) / kSThreads;
constexpr int kRedPerRow = kTX / 2 + 1;
constexpr int kBlackPerRow = kTX / 2;
constexpr int kOwn = kSTY * kTX / kSThreads;
constexpr int kCWX = kTX / 2 + 4;
constexpr int kCWY = kSTY / 2 + 4;
constexpr int kCCells = 2 * kCWX * kCWY;
constexpr int kCPer = (kCCells + kSThreads - 1) / kSThreads;
static_assert(kSTY * kTX % kSThreads == 0, "tile must be a multiple of the block");
static_assert((kSTY + 2) * kRedPerRow <= 2 * kSThreads, "at most two red nodes of the ring per thread");
static_assert(kWY * kCWX <= 2 * kSThreads, "at most two z-y interpolation entries per thread");


// Per-plane coefficients of planes base .. base+63, one plane per lane of
// every wave: the z-march reads plane p's value with a lane broadcast
// (v_readlane, the index is wave-uniform) instead of a scalar memory load
// whose wait would also hold up the LDS traffic of the step.
__device__ __forceinline__ float lane_bcast(float v, int lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ double lane_bcast(double v, int lane)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
struct PlaneTab {
    T v;
    int base;
    __device__ __forceinline__ void load(const MHS_CONST T *coef, int b, int comp, int nz)
    {
        base = b;
        const int p = b + (int)(threadIdx.x & 63);
        v = (p >= 0 && p < nz) ? coef[4 * p + comp] : (T)0;
    }
    __device__ __forceinline__ T operator()(int p) const { return lane_bcast(v, p - base); }
};

// LDS index pairs packed into one register (both < 65536).
__device__ __forceinline__ uint32_t pk16(int lo, int hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }
__device__ __forceinline__ int lo16(uint32_t v) { return (int)(v & 0xffffu); }
__device__ __forceinline__ int hi16(uint32_t v) { return (int)(v >> 16); }
// a or b by a 0/1 flag, as arithmetic (an indexed or selected register pair
// would be placed in scratch memory)
__device__ __forceinline__ uint32_t pick(uint32_t a, uint32_t b, int flag)
{
    return a ^ ((a ^ b) & (0u - (uint32_t)flag));
}
constexpr int kNone = 0xffff; // "no node" marker in a packed index

template <typename T, int FLAGS>
__global__ __launch_bounds__(kSThreads) MHS_SWEEP_ATTR void k_sweep3(const LevelItem *__restrict__ items, int nitems)
{
    constexpr bool HAS_F = (FLAGS & kHasF) != 0;
    constexpr bool ZERO_IN = (FLAGS & kZeroIn) != 0;
    constexpr bool NORM = (FLAGS & kNorm) != 0;
    constexpr bool PROLONG = (FLAGS & kProlong) != 0;
    // register-ring depth (planes of loads in flight); shallower when every
    // plane also carries right-hand-side or coarse-correction data
    constexpr int D = (HAS_F || PROLONG) ? kDepthF : kDepth;
    // the register classes of f (by plane parity) and the round of lcm(5, D)
    // steps are written for a ring of two planes
    static_assert(D == 2, "the smoother's march assumes a register ring of depth 2");
    constexpr int kCWPlanes = PROLONG ? 2 : 1;
    // right-hand-side values a thread reads per plane: its two red nodes,
    // its black node and, for the residual, its two own nodes
    constexpr int kNF = HAS_F ? (NORM ? 5 : 3) : 1;
    constexpr int kCPlane = kCWX * kCWY;
    // Window rows in LDS: even columns, then odd columns (half rows of HP
    // values), the odd half starting 16 banks after the even one.  The LDS
    // serves a wave's 32-bit accesses in half-waves of 32 lanes (measured: a
    // plain row layout, whose colour phases read every other word, raised
    // the bank-conflict cycles per LDS instruction of the FP32 sweep from
    // 1.37 to 1.80), so a half-wave reading or writing 32 nodes of one
    // colour in one row, or 32 consecutive cells of one row, is free of
    // conflicts.  With the row-aligned lane maps below the FP32 sweep has
    // 0.29 conflict cycles per LDS instruction (0.05 with stores masked off
    // for lanes without a cell, which cost more than they save); its time
    // is the same either way, so the LDS does not bound it.
    constexpr int HP = sizeof(T) == 8 ? MHS_SWEEP_HP64 : MHS_SWEEP_HP32;
    // FP32: the row pitch is 2 (mod 32) words, so that a half-wave spanning
    // several rows at the same columns (the last window columns, the last
    // red pair of the ring) spreads over the banks; the lane maps below keep
    // every other half-wave inside one row
    constexpr bool ROWMAP = sizeof(T) == 4 && MHS_SWEEP_ROWMAP32;
    constexpr int RW = sizeof(T) == 8 ? 2 * HP : MHS_SWEEP_RW32;
    constexpr int SLOT = kWY * RW;
    // (spare cells: kSpare takes the stores of lanes past the window; kTrash,
    // in row 1, the updates of lanes without a node, and every neighbour it
    // reads is a padding cell too)
    static_assert(HP >= kWX / 2 + 2 && RW >= HP + kWX / 2 + 1, "half row too short");
    constexpr int kSpare = RW - 1;
    constexpr int kTrash = RW + HP - 1;
    // five window slots: plane s+1 is staged while black(s-1) of the previous
    // step may still read planes s-2 .. s, so two barriers per step suffice
    constexpr int kSlots = 5;
    __shared__ T S[kSlots * SLOT];
    // Plane p lives in slot (p - kb + 2) % 5 (the right-hand side too, in
    // its own five slots).  The z-march runs in rounds of kRound steps, a
    // multiple of five and of the ring depth, so within a round every slot
    // and register set is a compile-time constant: LDS accesses take their
    // slot as an immediate offset and no step computes a modulo.
    constexpr int kRound = D % kSlots == 0 ? D : kSlots * D; // lcm(5, D) for D < 5
    static_assert(kRound % kSlots == 0 && kRound % D == 0, "round must cycle slots and ring");
    // every staged array has one spare cell past its data: lanes without a
    // cell store there, so staging is straight-line code (no divergent
    // branches between the loads and the stores that consume them)
    __shared__ T CW[kCWPlanes * kCPlane + 1];
    // prolongation: the coarse correction interpolated in z and y onto every
    // fine row of the window, at coarse columns (x interpolation at staging)
    __shared__ T ZW[PROLONG ? kWY * kCWX + 1 : 1];
    __shared__ double red[kSThreads / 64];
    auto sxp = [](int c) { return (c & 1) * HP + (c >> 1); };
    // Lane maps (FP32, row-aligned): window cell e -> (row, column): 64
    // consecutive columns per row, then the last kWX - 64 columns of every
    // row; red node e of the ring -> (row, pair q): 32 pairs per row, then
    // the last pair (q = kRedPerRow - 1) of every row.  (FP64: row-major.)
    auto cell_rc = [](int e, int &w, int &c) {
        if (!ROWMAP) {
            w = e / kWX;
            c = e - w * kWX;
        } else if (e < 64 * kWY) {
            w = e >> 6;
            c = e & 63;
        } else {
            const int x = e - 64 * kWY;
            w = x / (kWX - 64);
            c = 64 + x - w * (kWX - 64);
        }
    };
    auto red_wq = [](int e, int &w, int &q) {
        if (!ROWMAP) {
            w = 1 + e / kRedPerRow;
            q = e - (w - 1) * kRedPerRow;
        } else if (e < 32 * (kSTY + 2)) {
            w = 1 + (e >> 5);
            q = e & 31;
        } else {
            w = 1 + e - 32 * (kSTY + 2);
            q = kRedPerRow - 1;
        }
    };
    static_assert(!ROWMAP || (kRedPerRow == 33 && kWX - 64 == 4), "the row-aligned maps assume a 64-wide tile");

    const int tile = launch_tile(items, nitems);
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && gin<SolveState>(it->state)->done) return;
    const MHS_GLOBAL T *__restrict__ uin = gin<T>(it->u_in);
    MHS_GLOBAL T *__restrict__ uout = gout<T>(it->u_out);
    const MHS_GLOBAL T *__restrict__ f = gin<T>(it->f);
    const MHS_GLOBAL T *__restrict__ ec = gin<T>(it->ec);
    const MHS_CONST T *__restrict__ coef = gconst<T>(it->coef);
    const T cz = (T)it->cz;
    const int nx = it->nx, ny = it->ny, nz = it->nz;
    const int ncx = it->ncx, ncy = it->ncy, ncz = it->ncz;
    const int kz = it->kz;
    int local = tile - it->tile_base;
    const int tx = local % it->ntx;
    local /= it->ntx;
    const int ty = local % it->nty;
    const int tz = local / it->nty;
    const int i0 = 1 + tx * kTX, j0 = 1 + ty * kSTY;
    const int kb = 1 + tz * kz;
    const int ke = min(kb + kz, nz - 1);
    const int ptop = min(ke + 1, nz - 1); // highest plane read
    const size_t sxy = (size_t)nx * ny;
    const size_t csxy = (size_t)ncx * ncy;
    const int tid = threadIdx.x;
    const int I0 = (i0 - 2) >> 1, J0 = (j0 - 2) >> 1; // coarse window origin
    constexpr uint32_t es = sizeof(T);

    // ---- per-thread geometry, the same on every plane of the march --------
    // Window cells this thread stages: LDS index (kNone past the window) and
    // the ZW index of the cell's coarse column; byte offset of the clamped
    // in-plane source; inside-array, interior and odd-column flags.
    uint32_t st_i[kWPer];
    uint32_t st_g[kWPer];
    uint32_t st_in = 0, st_int = 0, st_odd = 0;
#pragma unroll
    for (int r = 0; r < kWPer; ++r) {
        const int e = tid + r * kSThreads;
        const int ee = min(e, kWCells - 1);
        int w, c;
        cell_rc(ee, w, c);
        const int i = i0 - 2 + c, j = j0 - 2 + w;
        st_i[r] = pk16(e < kWCells ? w * RW + sxp(c) : kSpare, PROLONG ? w * kCWX + ((i >> 1) - I0) : 0);
        st_g[r] = es * (uint32_t)(min(max(i, 0), nx - 1) + nx * min(max(j, 0), ny - 1));
        if (i >= 0 && i < nx && j >= 0 && j < ny) st_in |= 1u << r;
        if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) st_int |= 1u << r;
        if (i & 1) st_odd |= 1u << r;
    }
    // coarse-window cells (two coarse planes; LDS index tid + r * kSThreads)
    // and the z-y interpolation entries this thread computes
    uint32_t cw_g[PROLONG ? kCPer : 1];
    uint32_t cw_hi = 0;
    uint32_t zw_src = 0, zw_ok = 0, zw_odd = 0;
    if constexpr (PROLONG) {
#pragma unroll
        for (int r = 0; r < kCPer; ++r) {
            const int e = min(tid + r * kSThreads, kCCells - 1);
            const int pl = e / kCPlane;
            const int rem = e - pl * kCPlane;
            const int w = rem / kCWX, c = rem - w * kCWX;
            const int I = min(max(I0 + c, 0), ncx - 1), J = min(max(J0 + w, 0), ncy - 1);
            cw_g[r] = es * (uint32_t)(I + ncx * J);
            if (pl) cw_hi |= 1u << r;
        }
        int src[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int e = tid + r * kSThreads;
            const int ee = min(e, kWY * kCWX - 1);
            const int w = ee / kCWX, lc = ee - w * kCWX;
            const int j = j0 - 2 + w;
            src[r] = ((j >> 1) - J0) * kCWX + lc;
            if (e < kWY * kCWX) zw_ok |= 1u << r;
            if (j & 1) zw_odd |= 1u << r;
        }
        zw_src = pk16(src[0], src[1]);
    }
    // red nodes (tile plus a one-node ring) for each plane parity: centre
    // and west-neighbour indices (east = west + 1 in the colour-split row);
    // a lane whose node is not interior updates the padding cell kTrash
    uint32_t rd0[2], rd1[2];
    uint32_t rf[2][2]; // [plane parity][r]: byte offset of the node's f (clamped)
#pragma unroll
    for (int ps = 0; ps < 2; ++ps) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int e = tid + r * kSThreads;
            const int ee = min(e, (kSTY + 2) * kRedPerRow - 1);
            int w, q;
            red_wq(ee, w, q);
            const int c = 1 + ((ps + w) & 1) + 2 * q;
            const int i = i0 - 2 + c, j = j0 - 2 + w;
            const bool ok = e < (kSTY + 2) * kRedPerRow && i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2;
            const uint32_t v = ok ? pk16(w * RW + sxp(c), w * RW + sxp(c - 1)) : pk16(kTrash, kTrash - 1);
            if (ps)
                rd1[r] = v;
            else
                rd0[r] = v;
            rf[ps][r] = es * (uint32_t)(min(max(i, 0), nx - 1) + nx * min(max(j, 0), ny - 1));
        }
    }
    // black nodes of the tile (one per thread) for each plane parity
    uint32_t bk0 = 0, bk1 = 0;
    uint32_t bf[2]; // [plane parity]: byte offset of the black node's f (clamped)
    static_assert(kSTY * kBlackPerRow == kSThreads, "one black node per thread");
    {
#pragma unroll
        for (int ps = 0; ps < 2; ++ps) {
            const int w = 2 + tid / kBlackPerRow;
            const int q = tid - (w - 2) * kBlackPerRow;
            const int c = 2 + ((ps + w) & 1) + 2 * q;
            const int i = i0 - 2 + c, j = j0 - 2 + w;
            const uint32_t v = (i <= nx - 2 && j <= ny - 2) ? pk16(w * RW + sxp(c), w * RW + sxp(c - 1))
                                                            : pk16(kTrash, kTrash - 1);
            if (ps)
                bk1 = v;
            else
                bk0 = v;
            bf[ps] = es * (uint32_t)(min(i, nx - 1) + nx * min(j, ny - 1));
        }
    }
    // tile nodes this thread writes (and sums the residual of)
    uint32_t ow[kOwn];
    uint32_t ow_g[kOwn];
    uint32_t ow_ok = 0;
    static_assert(kOwn == 2, "two written nodes per thread");
    {
#pragma unroll
        for (int q = 0; q < kOwn; ++q) {
            const int e = tid + q * kSThreads;
            const int w = 2 + e / kTX, c = 2 + e % kTX;
            const int i = i0 + c - 2, j = j0 + w - 2;
            ow[q] = pk16(w * RW + sxp(c), w * RW + sxp(c - 1));
            // a node outside the interior gets an offset past the plane: its
            // buffer store is dropped (and a load there reads zero)
            const bool ok = i <= nx - 2 && j <= ny - 2;
            ow_g[q] = ok ? es * (uint32_t)(i + nx * j) : es * (uint32_t)sxy;
            if (ok) ow_ok |= 1u << q;
        }
    }
    const int par0 = (i0 + j0 + 1) & 1; // red parity of plane s is (par0 + s) & 1
    // waves holding a second red node (red nodes tid + kSThreads exist for
    // tid < (kSTY + 2) kRedPerRow - kSThreads); uniform per wave
    const bool two_red =
        __builtin_amdgcn_readfirstlane(tid) < (kSTY + 2) * kRedPerRow - kSThreads;
    // f offsets by plane class: class 0 = planes kb-1, kb+1, ...; class 1 =
    // planes kb, kb+2, ... (every step of the march knows its planes' class
    // at compile time)
    const int ps0 = (par0 + kb - 1) & 1;
    uint32_t fro[2][2], fbo[2]; // [class][r], [class]
#pragma unroll
    for (int cl = 0; cl < 2; ++cl) {
        const int ps = ps0 ^ cl;
        fro[cl][0] = pick(rf[0][0], rf[1][0], ps);
        fro[cl][1] = pick(rf[0][1], rf[1][1], ps);
        fbo[cl] = pick(bf[0], bf[1], ps);
    }
    // planes kb-1 .. ke (at most kKZ + 2 <= 64) of cx, cy, d, 1/d
    static_assert(kKZ + 2 <= 64, "one plane per lane");
    PlaneTab<T> tcx, tcy, tid_, tdd;
    tcx.load(coef, kb - 1, 0, nz);
    tcy.load(coef, kb - 1, 1, nz);
    tid_.load(coef, kb - 1, 3, nz);
    if constexpr (NORM) tdd.load(coef, kb - 1, 2, nz);

    auto at = [](const MHS_GLOBAL T *base, uint32_t byte_off) -> T {
        return *(const MHS_GLOBAL T *)((const MHS_GLOBAL char *)base + byte_off);
    };

    // Register ring: set q holds plane p's window (and right-hand side) and,
    // for the prolongation, the coarse data of plane p + 1, one plane ahead
    // so that its z-y interpolation can run during the red phase before the
    // plane is staged.
    T pre[D][kWPer];
    T fpre[D][kNF];
    T cpre[D][PROLONG ? kCPer : 1];
    // f of the planes in use: fcur = plane s (red, black, own), fbm = the
    // black node of plane s-1, fnx = plane s+1 (moved out of the ring when
    // the plane is staged)
    T fcur[kNF], fnx[kNF], fbm = (T)0;
#pragma unroll
    for (int k = 0; k < kNF; ++k) fcur[k] = fnx[k] = (T)0;
    // fine plane p lies between coarse planes p >> zs and (p + zs) >> zs
    // (zs = 0: the step kept z, and plane p has a coarse plane of its own)
    const int zs = ncz < nz ? 1 : 0;
    auto fetch_coarse = [&](int p, T(&cdst)[PROLONG ? kCPer : 1]) {
        if constexpr (PROLONG) {
            const MHS_GLOBAL T *p0 = ec + csxy * (size_t)min(p >> zs, ncz - 1);
            const MHS_GLOBAL T *p1 = ec + csxy * (size_t)min((p + zs) >> zs, ncz - 1);
#pragma unroll
            for (int r = 0; r < kCPer; ++r) cdst[r] = at(((cw_hi >> r) & 1) ? p1 : p0, cw_g[r]);
        }
    };
    // Loads are unconditional, from clamped in-bounds addresses, straight
    // into the ring registers; cells outside the array are zeroed when the
    // plane is staged.
    const uint32_t plane_bytes = es * (uint32_t)sxy;
    // cl: the class of plane p (its colour layout)
    auto fetch = [&](int p, int cl, T(&dst)[kWPer], T(&fdst)[kNF], T(&cdst)[PROLONG ? kCPer : 1]) {
        if constexpr (!ZERO_IN) {
            const auto rs = plane_rsrc(uin + sxy * (size_t)p, plane_bytes);
#pragma unroll
            for (int r = 0; r < kWPer; ++r) dst[r] = bload<T>(rs, st_g[r]);
        }
        if constexpr (HAS_F) {
            const auto rs = plane_rsrc(f + sxy * (size_t)p, plane_bytes);
            fdst[0] = bload<T>(rs, cl ? fro[1][0] : fro[0][0]);
            fdst[1] = bload<T>(rs, cl ? fro[1][1] : fro[0][1]);
            fdst[2] = bload<T>(rs, cl ? fbo[1] : fbo[0]);
            if constexpr (NORM) {
                fdst[3] = bload<T>(rs, ow_g[0]);
                fdst[4] = bload<T>(rs, ow_g[1]);
            }
        }
        fetch_coarse(p + 1, cdst);
    };
    auto store_cw = [&](const T(&csrc)[PROLONG ? kCPer : 1]) {
        if constexpr (PROLONG) {
#pragma unroll
            for (int r = 0; r < kCPer; ++r) CW[min(tid + r * kSThreads, kCCells)] = csrc[r];
        }
    };
    // z-y interpolation of the staged coarse planes for fine plane p
    auto zy_rows = [&](int p) {
        if constexpr (PROLONG) {
            const T h = (T)0.5;
            const bool ok = (p & zs) != 0;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                {
                    const int a = r ? hi16(zw_src) : lo16(zw_src);
                    const bool oj = (zw_odd >> r) & 1;
                    const T a0 = CW[a], y0 = oj ? h * (a0 + CW[a + kCWX]) : a0;
                    T v = y0;
                    if (ok) {
                        const T a1 = CW[kCPlane * (kCWPlanes - 1) + a];
                        const T y1 = oj ? h * (a1 + CW[kCPlane * (kCWPlanes - 1) + a + kCWX]) : a1;
                        v = h * (y0 + y1);
                    }
                    ZW[(zw_ok >> r) & 1 ? tid + r * kSThreads : kWY * kCWX] = v;
                }
            }
        }
    };
    // stage plane p (window with the coarse correction from ZW, right-hand
    // side) and the coarse planes of p + 1 carried by the same register set
    auto stash = [&](int p, int sl, const T(&src)[kWPer], const T(&fsrc)[kNF],
                     const T(&csrc)[PROLONG ? kCPer : 1]) {
        const bool corr = PROLONG && p >= 1 && p <= nz - 2;
        T *dst = S + sl * SLOT;
#pragma unroll
        for (int r = 0; r < kWPer; ++r) {
            const int l = lo16(st_i[r]); // kSpare (a padding cell) past the window
            T v = (!ZERO_IN && ((st_in >> r) & 1)) ? src[r] : (T)0;
            if constexpr (PROLONG) {
                if (corr && ((st_int >> r) & 1)) {
                    const int z = hi16(st_i[r]);
                    const T a = ZW[z];
                    v += ((st_odd >> r) & 1) ? (T)0.5 * (a + ZW[z + 1]) : a;
                }
            }
            dst[l] = v;
        }
        if constexpr (HAS_F) {
#pragma unroll
            for (int k = 0; k < kNF; ++k) fnx[k] = fsrc[k];
        }
        store_cw(csrc);
    };

    // tile nodes of plane m from LDS to u_out
    auto write_plane = [&](int m, int sl) {
        const T *P = S + sl * SLOT;
        const auto rs = plane_rsrc(uout + sxy * (size_t)m, plane_bytes);
#pragma unroll
        for (int q = 0; q < kOwn; ++q) bstore(P[lo16(ow[q])], rs, ow_g[q]);
    };

    double acc = 0.0;
    T below[kOwn];
#pragma unroll
    for (int q = 0; q < kOwn; ++q) below[q] = (T)0;

    // plane p waits in register set (p - pbase) % D until it is staged;
    // its class (for the f offsets) is (p - kb + 1) & 1
    const int pbase = kb - 2;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        const int p = pbase + q;
        fetch(min(max(p, 0), ptop), (q + 1) & 1, pre[q], fpre[q], cpre[q]);
    }
    // warm-up: stage planes kb-2 (if any) and kb-1; the prolongation needs
    // the z-y rows of each plane ready before it is staged
    if constexpr (PROLONG) {
        const int pf = max(pbase, 0);
        T c0[kCPer];
        fetch_coarse(pf, c0);
        store_cw(c0);
        lds_barrier();
        zy_rows(pf);
        lds_barrier();
    }
    if (pbase >= 0) {
        stash(pbase, 0, pre[0], fpre[0], cpre[0]);
        if constexpr (PROLONG) {
            lds_barrier();
            zy_rows(pbase + 1);
            lds_barrier();
        }
    }
    stash(kb - 1, 1, pre[1], fpre[1], cpre[1]);
    if constexpr (PROLONG) {
        lds_barrier();
        zy_rows(kb);
        lds_barrier();
    }
#pragma unroll
    for (int k = 0; k < kNF; ++k) fcur[k] = fnx[k]; // f of plane kb-1
    // the two sets in issue order, as the steps issue them (interleaved, the
    // first wait of every round would have to cover both)
    fetch(min(pbase + D, ptop), (D + 1) & 1, pre[0], fpre[0], cpre[0]);
    __builtin_amdgcn_sched_barrier(0);
    fetch(min(pbase + D + 1, ptop), D & 1, pre[1], fpre[1], cpre[1]);
    __builtin_amdgcn_sched_barrier(0);

    // One step: stage plane s+1, red of plane s, black of plane s-1, write
    // of plane s-2.  ri is the register set of plane s+1; sm2 .. sp1 are the
    // slots of planes s-2 .. s+1; d is the step's position in its round
    // (its parity gives the class of the plane it fetches).
    auto step = [&](const int s, const int d, const int ri, const int sm2, const int sm1, const int s00,
                    const int sp1) {
        // stage plane s+1 (slot of plane s-4; the previous step's black
        // phase may still read planes s-3 .. s-1) and refill its register
        // set with plane s+1+D.  Both are unconditional (past the top of
        // the chunk they repeat the last plane, and a stage of plane nz
        // lands in a slot no phase reads) so that every step issues the
        // same loads and the compiler can wait for the oldest set only.
        stash(s + 1, sp1, pre[ri], fpre[ri], cpre[ri]);
        fetch(min(s + 1 + D, ptop), (d + D + 1) & 1, pre[ri], fpre[ri], cpre[ri]);
        // keep each step's loads in its step (moved across steps, the
        // waits of the next stage would cover the wrong register set)
        __builtin_amdgcn_sched_barrier(0);
        lds_barrier();
        const T *Ps = S + s00 * SLOT;
        const T *Pu = S + sp1 * SLOT;
        const T *Pd = S + sm1 * SLOT;
        if constexpr (NORM) {
            // residual of the input iterate at plane s (all values still
            // old); old plane s-1 comes from registers captured a step ago
            const bool do_res = (s >= kb && s < ke);
            T cx = 0, cy = 0, dd = 0;
            if (do_res) {
                cx = tcx(s);
                cy = tcy(s);
                dd = tdd(s);
            }
#pragma unroll
            for (int q = 0; q < kOwn; ++q) {
                const int o = lo16(ow[q]), ww = hi16(ow[q]);
                const T uc = Ps[o];
                if (do_res && ((ow_ok >> q) & 1)) {
                    T fv = (T)0;
                    if constexpr (HAS_F) fv = fcur[3 + q];
                    const T r = fv - (cx * (Ps[ww + 1] + Ps[ww]) + cy * (Ps[o + RW] + Ps[o - RW]) +
                                      cz * (Pu[o] + below[q]) + dd * uc);
                    acc += (double)r * (double)r;
                }
                below[q] = uc;
            }
            lds_barrier();
        }
        // z-y rows of plane s+2, whose coarse planes were staged with s+1
        zy_rows(s + 2);
        // write plane s-2, final since black(s-2) ended before the barrier
        if (s - 2 >= kb && s - 2 < ke) write_plane(s - 2, sm2);
        // red nodes of plane s on the tile and its one-node ring
        if (s >= 1 && s <= nz - 2) {
            const T cx = tcx(s), cy = tcy(s), invd = tid_(s);
            T *P = S + s00 * SLOT;
            const int ps = (par0 + s) & 1;
            // the second red node exists only for the first waves (the
            // ring has more red nodes than the workgroup has threads): a
            // wave-uniform choice, with both nodes' reads issued together
            auto red = [&](int nr) {
                int o[2], ww[2];
                T v[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    if (r >= nr) break;
                    const uint32_t pr = pick(rd0[r], rd1[r], ps);
                    o[r] = lo16(pr);
                    ww[r] = hi16(pr);
                    T fv = (T)0;
                    if constexpr (HAS_F) fv = fcur[r];
                    v[r] = (fv - (cx * (P[ww[r] + 1] + P[ww[r]]) + cy * (P[o[r] + RW] + P[o[r] - RW]) +
                                  cz * (Pu[o[r]] + Pd[o[r]]))) *
                           invd;
                }
#pragma unroll
                for (int r = 0; r < 2; ++r)
                    if (r < nr) P[o[r]] = v[r];
            };
            if (two_red)
                red(2);
            else
                red(1);
        }
        lds_barrier();
        // black nodes of plane m = s - 1 on the tile
        const int m = s - 1;
        if (m >= kb && m < ke) {
            const T cx = tcx(m), cy = tcy(m), invd = tid_(m);
            T *P = S + sm1 * SLOT;
            const T *Pm = S + sm2 * SLOT;
            const int pb = (par0 + m) & 1;
            const uint32_t pr = pick(bk0, bk1, pb);
            const int o = lo16(pr);
            const int ww = hi16(pr);
            T fv = (T)0;
            if constexpr (HAS_F) fv = fbm;
            P[o] = (fv - (cx * (P[ww + 1] + P[ww]) + cy * (P[o + RW] + P[o - RW]) + cz * (Ps[o] + Pm[o]))) * invd;
        }
        // f of the next step: black of plane s, all of plane s+1
        if constexpr (HAS_F) {
            fbm = fcur[2];
#pragma unroll
            for (int k = 0; k < kNF; ++k) fcur[k] = fnx[k];
        }
    };
    // Whole rounds with constant slots and register sets (no exit inside a
    // round: an early exit would add paths into later steps on which the
    // newest loads belong to another set, and the compiler's waits would
    // then drain the ring), then the remaining steps with slots computed.
    int s0 = kb - 1;
    for (; s0 + kRound - 1 <= ke; s0 += kRound) {
#pragma unroll
        for (int d = 0; d < kRound; ++d)
            step(s0 + d, d, (d + 2) % D, (d + 4) % kSlots, d % kSlots, (d + 1) % kSlots, (d + 2) % kSlots);
    }
    for (; s0 <= ke; s0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int s = s0 + d;
            if (s > ke) break;
            const int t = s - kb + 2; // slot of plane s
            step(s, d, (d + 2) % D, (t + 3) % kSlots, (t + 4) % kSlots, t % kSlots, (t + 1) % kSlots);
        }
    }
    // the last planes: ke-2 was written in the final step, ke-1 remains
    lds_barrier();
    if (ke - 1 >= kb) write_plane(ke - 1, (ke - kb + 1) % kSlots);
    if constexpr (NORM) {
        const double tot = block_sum<kSThreads>(acc, red);
        if (tid == 0) gout<double>(it->partials)[tile - it->tile_base] = tot;
    }
}

// ============================================================================
// 2D red-black sweeps for equation (11): one plane, ping-pong; one or two
// complete sweeps per launch (kTwoSweeps).  A workgroup stages its
// kTX x kTY2 tile plus a halo of two nodes per sweep, and sweep s updates
// the red nodes of the tile and a ring of 2 (NS - s) - 1 nodes, then the
// black nodes of the tile and a ring of 2 (NS - s) - 2: every value the
// tile's last black update reads is then final, as in the sweeps done one
// launch at a time, and a ring node computed by two workgroups gets the
// same value in both.  Two sweeps per launch cost one launch instead of two
// on these small, launch-bound planes.
// ============================================================================
constexpr int kOwn2 = kTY2 * kTX / kThreads;
static_assert(kTY2 * kTX % kThreads == 0, "tile must be a multiple of the block");

template <typename T, int FLAGS>
__global__ __launch_bounds__(kThreads) void k_sweep2(const LevelItem *__restrict__ items, int nitems)
{
    constexpr bool HAS_F = (FLAGS & kHasF) != 0;
    constexpr bool ZERO_IN = (FLAGS & kZeroIn) != 0;
    constexpr bool NORM = (FLAGS & kNorm) != 0;
    constexpr bool PROLONG = (FLAGS & kProlong) != 0;
    constexpr int NS = (FLAGS & kTwoSweeps) ? 2 : 1;
    constexpr int H = 2 * NS; // halo
    constexpr int WX = kTX + 2 * H, WY = kTY2 + 2 * H;
    __shared__ T S[WY][WX];
    __shared__ double red[kThreads / 64];

    const int tile = launch_tile(items, nitems);
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && gin<SolveState>(it->state)->done) return;
    const MHS_GLOBAL T *__restrict__ uin = gin<T>(it->u_in);
    MHS_GLOBAL T *__restrict__ uout = gout<T>(it->u_out);
    const MHS_GLOBAL T *__restrict__ f = gin<T>(it->f);
    const MHS_GLOBAL T *__restrict__ ec = gin<T>(it->ec);
    const MHS_CONST T *__restrict__ coef = gconst<T>(it->coef);
    const int nx = it->nx, ny = it->ny;
    const int ncx = it->ncx;
    const int local = tile - it->tile_base;
    const int tx = local % it->ntx, ty = local / it->ntx;
    const int i0 = 1 + tx * kTX, j0 = 1 + ty * kTY2;
    const int tid = threadIdx.x;
    const T cx = coef[0], cy = coef[1], d = coef[2], invd = coef[3];

    // window cell (w, c) is node (i0 - H + c, j0 - H + w)
    for (int e = tid; e < WY * WX; e += kThreads) {
        const int w = e / WX, c = e - w * WX;
        const int i = i0 - H + c, j = j0 - H + w;
        T v = (T)0;
        if (i >= 0 && i < nx && j >= 0 && j < ny) {
            if constexpr (!ZERO_IN) v = uin[(size_t)i + (size_t)nx * j];
            if constexpr (PROLONG) {
                if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) v += interp2<T>(ec, ncx, i, j);
            }
        }
        S[w][c] = v;
    }
    lds_barrier();
    double acc = 0.0;
    if constexpr (NORM) {
#pragma unroll
        for (int q = 0; q < kOwn2; ++q) {
            const int e = tid + q * kThreads;
            const int w = H + e / kTX, c = H + e % kTX;
            const int i = i0 + c - H, j = j0 + w - H;
            if (i <= nx - 2 && j <= ny - 2) {
                T fv = (T)0;
                if constexpr (HAS_F) fv = f[(size_t)i + (size_t)nx * j];
                const T r = fv - (cx * (S[w][c + 1] + S[w][c - 1]) + cy * (S[w + 1][c] + S[w - 1][c]) + d * S[w][c]);
                acc += (double)r * (double)r;
            }
        }
        lds_barrier();
    }
    // nodes of colour p ((i + j) & 1, red = 0) on the tile and a ring of r
    // nodes: (kTY2 + 2r) rows of kTX/2 + r nodes each
    auto colour = [&](int p, int r) {
        const int per_row = kTX / 2 + r;
        for (int e = tid; e < (kTY2 + 2 * r) * per_row; e += kThreads) {
            const int rr = e / per_row;
            const int q = e - rr * per_row;
            const int w = H - r + rr;
            const int j = j0 - H + w;
            const int c0 = H - r;
            const int c = c0 + ((p - j - (i0 - H) - c0) & 1) + 2 * q;
            const int i = i0 - H + c;
            if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) {
                T fv = (T)0;
                if constexpr (HAS_F) fv = f[(size_t)i + (size_t)nx * j];
                S[w][c] = (fv - (cx * (S[w][c + 1] + S[w][c - 1]) + cy * (S[w + 1][c] + S[w - 1][c]))) * invd;
            }
        }
    };
#pragma unroll
    for (int sw = 0; sw < NS; ++sw) {
        colour(0, 2 * (NS - sw) - 1);
        lds_barrier();
        colour(1, 2 * (NS - sw) - 2);
        lds_barrier();
    }
    for (int e = tid; e < kTY2 * kTX; e += kThreads) {
        const int w = H + e / kTX, c = H + e % kTX;
        const int i = i0 + c - H, j = j0 + w - H;
        if (i <= nx - 2 && j <= ny - 2) uout[(size_t)i + (size_t)nx * j] = S[w][c];
    }
    if constexpr (NORM) {
        const double tot = block_sum<kThreads>(acc, red);
        if (tid == 0) gout<double>(it->partials)[tile - it->tile_base] = tot;
    }
}

// ============================================================================
// 3D residual r = f - A u (on the fly) + full weighting onto coarse nodes:
//   f_c(I,J,K) = sum_{a,b,c in -1..1} w_a w_b w_c r(2I+a, 2J+b, 2K+c),
//   w_0 = 1/2, w_{+-1} = 1/4,
// or, on a step that keeps z (x-y semicoarsening), the same weights within
// each plane: f_c(I,J,k) = sum_{a,b} w_a w_b r(2I+a, 2J+b, k).
// A workgroup owns kCX x kCY coarse nodes and marches kKC coarse planes; each
// fine plane's residual is computed once into LDS from an LDS-staged window
// of u (three planes in flight) and folded into the coarse sums.
// ============================================================================
constexpr int kRWX = 2 * kCX + 3;
constexpr int kRWY = 2 * kCY + 3;
constexpr int kRRX = 2 * kCX + 1;
constexpr int kRRY = 2 * kCY + 1;
static_assert(kCX * kCY == kThreads, "one coarse node per thread");

template <typename T, bool HAS_F, bool KEEPZ>
__global__ __launch_bounds__(kThreads) void k_restrict3(const LevelItem *__restrict__ items, int nitems)
{
    constexpr int kCells = kRWY * kRWX;
    constexpr int kPer = (kCells + kThreads - 1) / kThreads;
    constexpr int kRCells = kRRY * kRRX;
    constexpr int kRPer = (kRCells + kThreads - 1) / kThreads;
    constexpr int D = HAS_F ? 3 : kDepth;
    constexpr int USLOT = kRWY * kRWX;
    __shared__ T U[4 * USLOT];
    __shared__ T R[kRCells];

    const int tile = launch_tile(items, nitems);
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && gin<SolveState>(it->state)->done) return;
    const MHS_GLOBAL T *__restrict__ u = gin<T>(it->u_in);
    const MHS_GLOBAL T *__restrict__ f = gin<T>(it->f);
    MHS_GLOBAL T *__restrict__ fc = gout<T>(it->u_out);
    const MHS_CONST T *__restrict__ coef = gconst<T>(it->coef);
    const T cz = (T)it->cz;
    const int nx = it->nx, ny = it->ny;
    const int ncx = it->ncx, ncy = it->ncy, ncz = it->ncz;
    const int kc = it->kz;
    int local = tile - it->tile_base;
    const int tx = local % it->ntx;
    local /= it->ntx;
    const int ty = local % it->nty;
    const int tz = local / it->nty;
    const int I0 = 1 + tx * kCX, J0 = 1 + ty * kCY;
    const int Kb = 1 + tz * kc;
    const int Ke = min(Kb + kc, ncz - 1);
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1; // residual window origin
    const int ui0 = fi0 - 1, uj0 = fj0 - 1;       // u window origin
    const size_t sxy = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const int tI = tid % kCX, tJ = tid / kCX;
    const int I = I0 + tI, J = J0 + tJ;
    const bool valid = (I <= ncx - 2) && (J <= ncy - 2);
    constexpr uint32_t es = sizeof(T);

    // ---- per-thread geometry, fixed for the whole z-march ------------------
    // u window cells staged by this thread
    int st_l[kPer];
    uint32_t st_g[kPer];
    uint32_t st_in = 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int e = tid + r * kThreads;
        const int ee = min(e, kCells - 1);
        const int w = ee / kRWX, c = ee - w * kRWX;
        const int i = ui0 + c, j = uj0 + w;
        st_l[r] = e < kCells ? ee : -1;
        st_g[r] = es * (uint32_t)(min(max(i, 0), nx - 1) + nx * min(max(j, 0), ny - 1));
        if (i < nx && j < ny) st_in |= 1u << r;
    }
    // residual cells this thread computes: U centre and R index, interior
    // flag, byte offset of f
    uint32_t rc[kRPer];
    uint32_t rc_g[HAS_F ? kRPer : 1];
    uint32_t rc_int = 0;
#pragma unroll
    for (int r = 0; r < kRPer; ++r) {
        const int e = tid + r * kThreads;
        const int ee = min(e, kRCells - 1);
        const int w = ee / kRRX, c = ee - w * kRRX;
        const int i = fi0 + c, j = fj0 + w;
        rc[r] = pk16((w + 1) * kRWX + (c + 1), e < kRCells ? ee : kNone);
        if constexpr (HAS_F) rc_g[r] = es * (uint32_t)(min(i, nx - 1) + nx * min(j, ny - 1));
        if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) rc_int |= 1u << r;
    }
    const uint32_t out_g = es * (uint32_t)(min(I, ncx - 1) + ncx * min(J, ncy - 1));
    const size_t csxy = (size_t)ncx * ncy;

    auto at = [](const MHS_GLOBAL T *base, uint32_t byte_off) -> T {
        return *(const MHS_GLOBAL T *)((const MHS_GLOBAL char *)base + byte_off);
    };
    // register set q holds u plane p and f plane p - 1 (the residual plane
    // computed in the step that stages u plane p)
    T pre[D][kPer];
    T fpre[D][HAS_F ? kRPer : 1];
    auto fetch = [&](int p, T(&dst)[kPer], T(&fdst)[HAS_F ? kRPer : 1]) {
        const MHS_GLOBAL T *pl = u + sxy * (size_t)p;
#pragma unroll
        for (int r = 0; r < kPer; ++r) dst[r] = at(pl, st_g[r]);
        if constexpr (HAS_F) {
            const MHS_GLOBAL T *fl = f + sxy * (size_t)max(p - 1, 0);
#pragma unroll
            for (int r = 0; r < kRPer; ++r) fdst[r] = at(fl, rc_g[r]);
        }
    };
    auto stash = [&](int p, const T(&src)[kPer]) {
        T *dst = U + (p & 3) * USLOT;
#pragma unroll
        for (int r = 0; r < kPer; ++r)
            if (st_l[r] >= 0) dst[st_l[r]] = ((st_in >> r) & 1) ? src[r] : (T)0;
    };

    // residual planes mfirst .. mlast (2Kb-1 .. 2Ke-1, or Kb .. Ke-1 when z
    // is kept) from u planes mfirst-1 .. mlast+1; plane p waits in register
    // set (p - pbase) % D.  Every step issues the same loads (past the top
    // they repeat the last plane), so the compiler waits for exactly the
    // oldest register set.
    const int mfirst = KEEPZ ? Kb : 2 * Kb - 1, mlast = KEEPZ ? Ke - 1 : 2 * Ke - 1;
    const int pbase = mfirst - 1, ptop = mlast + 1;
    // the residual planes' cx, cy, d (at most 2 kKC + 1 <= 64)
    static_assert(2 * kKC + 1 <= 64, "one plane per lane");
    PlaneTab<T> tcx, tcy, tdd;
    tcx.load(coef, mfirst, 0, it->nz);
    tcy.load(coef, mfirst, 1, it->nz);
    tdd.load(coef, mfirst, 2, it->nz);
#pragma unroll
    for (int q = 0; q < D; ++q) {
        fetch(min(pbase + q, ptop), pre[q], fpre[q]);
        __builtin_amdgcn_sched_barrier(0);
    }
    stash(pbase, pre[0]);
    stash(pbase + 1, pre[1]);
    fetch(min(pbase + D, ptop), pre[0], fpre[0]);
    __builtin_amdgcn_sched_barrier(0);
    fetch(min(pbase + D + 1, ptop), pre[1], fpre[1]);
    __builtin_amdgcn_sched_barrier(0);
    T acc = (T)0;
    const T q4 = (T)0.25, h2 = (T)0.5;
    const int cw = 2 * tJ + 1, cc = 2 * tI + 1;
    // whole rounds of D steps (one back edge, so the compiler's waits hold
    // only the oldest register set); a step past mlast only stages and
    // fetches
    for (int m0 = mfirst; m0 <= mlast; m0 += D) {
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            const int m = m0 + dd;
            const bool live = m <= mlast;
            // stage u plane m+1 into the slot of plane m-3 (read two steps
            // ago); its register set also carries f plane m
            const int ri = (dd + 2) % D;
            stash(m + 1, pre[ri]);
            lds_barrier();
            if (live) {
                const T cx = tcx(m), cy = tcy(m), d = tdd(m);
                const T *P = U + (m & 3) * USLOT;
                const T *Pm = U + ((m - 1) & 3) * USLOT;
                const T *Pp = U + ((m + 1) & 3) * USLOT;
#pragma unroll
                for (int r = 0; r < kRPer; ++r) {
                    const int ri_ = hi16(rc[r]);
                    if (ri_ == kNone) continue;
                    const int o = lo16(rc[r]);
                    T rv = (T)0;
                    if ((rc_int >> r) & 1) {
                        T fv = (T)0;
                        if constexpr (HAS_F) fv = fpre[ri][r];
                        rv = fv - (cx * (P[o + 1] + P[o - 1]) + cy * (P[o + kRWX] + P[o - kRWX]) +
                                   cz * (Pp[o] + Pm[o]) + d * P[o]);
                    }
                    R[ri_] = rv;
                }
            }
            fetch(min(m + 1 + D, ptop), pre[ri], fpre[ri]);
            lds_barrier();
            if (!live) continue;
            auto row = [&](int w) {
                return q4 * R[w * kRRX + cc - 1] + h2 * R[w * kRRX + cc] + q4 * R[w * kRRX + cc + 1];
            };
            const T s2 = q4 * row(cw - 1) + h2 * row(cw) + q4 * row(cw + 1);
            if constexpr (KEEPZ) {
                if (valid) *(MHS_GLOBAL T *)((MHS_GLOBAL char *)(fc + csxy * (size_t)m) + out_g) = s2;
            } else if (m & 1) {
                const int Kend = (m - 1) >> 1;
                if (Kend >= Kb) {
                    acc += q4 * s2;
                    if (valid) *(MHS_GLOBAL T *)((MHS_GLOBAL char *)(fc + csxy * (size_t)Kend) + out_g) = acc;
                }
                acc = q4 * s2;
            } else {
                acc += h2 * s2;
            }
        }
    }
}


// ============================================================================
// Steps that keep x and y (z semicoarsening, for grids with dz well below dx
// and dy): residual + full weighting along z, and the correction's linear
// interpolation along z.  One thread per coarse (restriction) or fine
// (prolongation) interior node, reads through the caches; such levels are
// rare and small, so these kernels favour plainness over the tiled march.
// ============================================================================
template <typename T, bool HAS_F>
__global__ __launch_bounds__(kThreads) void k_restrict3_z(const LevelItem *__restrict__ items, int nitems)
{
    const int tile = launch_tile(items, nitems);
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && gin<SolveState>(it->state)->done) return;
    const int nx = it->nx, ny = it->ny, ncz = it->ncz;
    const int mx = nx - 2, my = ny - 2;
    const int64_t e = (int64_t)(tile - it->tile_base) * kThreads + threadIdx.x;
    if (e >= (int64_t)mx * my * (ncz - 2)) return;
    const int i = 1 + (int)(e % mx);
    const int64_t q = e / mx;
    const int j = 1 + (int)(q % my), K = 1 + (int)(q / my);
    const MHS_GLOBAL T *__restrict__ u = gin<T>(it->u_in);
    const MHS_GLOBAL T *__restrict__ f = gin<T>(it->f);
    MHS_GLOBAL T *__restrict__ fc = gout<T>(it->u_out);
    const MHS_CONST T *__restrict__ coef = gconst<T>(it->coef);
    const T cz = (T)it->cz;
    const size_t sxy = (size_t)nx * ny, col = (size_t)i + (size_t)nx * j;
    T acc = (T)0;
#pragma unroll
    for (int c = -1; c <= 1; ++c) {
        const int k = 2 * K + c; // 1 <= k <= nz - 2
        const size_t o = col + sxy * k;
        const T cx = coef[4 * k], cy = coef[4 * k + 1], d = coef[4 * k + 2];
        const T fv = HAS_F ? f[o] : (T)0;
        const T rv = fv - (cx * (u[o + 1] + u[o - 1]) + cy * (u[o + nx] + u[o - nx]) + cz * (u[o + sxy] + u[o - sxy]) +
                           d * u[o]);
        acc += (c == 0 ? (T)0.5 : (T)0.25) * rv;
    }
    fc[col + sxy * K] = acc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_prolong3_z(const LevelItem *__restrict__ items, int nitems)
{
    const int tile = launch_tile(items, nitems);
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && gin<SolveState>(it->state)->done) return;
    const int nx = it->nx, ny = it->ny, nz = it->nz;
    const int mx = nx - 2, my = ny - 2;
    const int64_t e = (int64_t)(tile - it->tile_base) * kThreads + threadIdx.x;
    if (e >= (int64_t)mx * my * (nz - 2)) return;
    const int i = 1 + (int)(e % mx);
    const int64_t q = e / mx;
    const int j = 1 + (int)(q % my), k = 1 + (int)(q / my);
    const MHS_GLOBAL T *__restrict__ ec = gin<T>(it->ec);
    MHS_GLOBAL T *__restrict__ u = gout<T>(it->u_out);
    const size_t sxy = (size_t)nx * ny, col = (size_t)i + (size_t)nx * j;
    const size_t c0 = col + sxy * (size_t)(k >> 1); // coarse plane k/2 (x, y kept)
    const T v = (k & 1) ? (T)0.5 * ec[c0] + (T)0.5 * ec[c0 + sxy] : ec[c0];
    u[col + sxy * k] += v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict2(const LevelItem *__restrict__ items, int nitems)
{
    __shared__ T U[kRWY][kRWX];
    __shared__ T R[kRRY][kRRX];
    const int tile = launch_tile(items, nitems);
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && gin<SolveState>(it->state)->done) return;
    const MHS_GLOBAL T *__restrict__ u = gin<T>(it->u_in);
    const MHS_GLOBAL T *__restrict__ f = gin<T>(it->f);
    MHS_GLOBAL T *__restrict__ fc = gout<T>(it->u_out);
    const MHS_CONST T *__restrict__ coef = gconst<T>(it->coef);
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
    lds_barrier();
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
    lds_barrier();
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
constexpr int kICells = kIWX * kIWY;
constexpr int kIPer = (kICells + kThreads - 1) / kThreads;

template <bool HAS_E, bool ZERO_IN>
__global__ __launch_bounds__(kThreads) void k_ir3(const LevelItem *__restrict__ items, int nitems)
{
    constexpr int D = kDepth;
    constexpr int SLOT = kIWY * kIWX + 1; // one spare cell: stores of lanes past the window
    constexpr int kOwnI = kTY * kTX / kThreads;
    // four slots; the march runs in rounds of four steps (a multiple of the
    // ring depth), so within a round every slot is a compile-time constant
    constexpr int kSlotsI = 4;
    constexpr int kRoundI = 4;
    static_assert(kRoundI % D == 0, "round must cycle the ring");
    __shared__ double S[kSlotsI * SLOT];
    __shared__ double red[kThreads / 64];
    const int tile = launch_tile(items, nitems);
    const LevelItem *it = items + find_item(items, nitems, tile);
    if (it->state && gin<SolveState>(it->state)->done) return;
    const MHS_GLOBAL double *__restrict__ uin = gin<double>(it->u_in);
    MHS_GLOBAL double *__restrict__ uout = gout<double>(it->u_out);
    const MHS_GLOBAL float *__restrict__ e32 = gin<float>(it->ec);
    MHS_GLOBAL float *__restrict__ r32 = gout<float>(it->r_out);
    const MHS_CONST double *__restrict__ coef = gconst<double>(it->coef);
    const double cz = it->cz;
    const int nx = it->nx, ny = it->ny, nz = it->nz;
    const int kz = it->kz;
    int local = tile - it->tile_base;
    const int tx = local % it->ntx;
    local /= it->ntx;
    const int ty = local % it->nty;
    const int tz = local / it->nty;
    const int i0 = 1 + tx * kTX, j0 = 1 + ty * kTY;
    const int kb = 1 + tz * kz;
    const int ke = min(kb + kz, nz - 1);
    const size_t sxy = (size_t)nx * ny;
    const uint32_t plane_elems = (uint32_t)sxy;
    const int tid = threadIdx.x;

    // ---- per-thread geometry, fixed for the whole z-march ------------------
    // window cells staged: LDS index (the spare cell past the window), byte
    // offsets of the clamped source in an FP64 and an FP32 plane, inside-
    // array and interior flags
    int st_l[kIPer];
    uint32_t st_g[kIPer];
    uint32_t st_in = 0, st_int = 0;
#pragma unroll
    for (int r = 0; r < kIPer; ++r) {
        const int e = tid + r * kThreads;
        const int ee = min(e, kICells - 1);
        const int w = ee / kIWX, c = ee - w * kIWX;
        const int i = i0 - 1 + c, j = j0 - 1 + w;
        st_l[r] = e < kICells ? ee : SLOT - 1;
        st_g[r] = (uint32_t)(min(max(i, 0), nx - 1) + nx * min(max(j, 0), ny - 1));
        if (i < nx && j < ny) st_in |= 1u << r;
        if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) st_int |= 1u << r;
    }
    // tile nodes this thread updates: LDS index and element offset; a node
    // outside the array gets an offset past the end of the plane, where the
    // buffer store is dropped
    int ow_l[kOwnI];
    uint32_t ow_g[kOwnI];
    uint32_t ow_ok = 0;
#pragma unroll
    for (int q = 0; q < kOwnI; ++q) {
        const int e = tid + q * kThreads;
        const int w = 1 + e / kTX, c = 1 + e % kTX;
        const int i = i0 + c - 1, j = j0 + w - 1;
        const bool ok = i <= nx - 2 && j <= ny - 2;
        ow_l[q] = w * kIWX + c;
        ow_g[q] = ok ? (uint32_t)(i + nx * j) : plane_elems;
        if (ok) ow_ok |= 1u << q;
    }

    double pre[D][kIPer];
    float epre[D][HAS_E ? kIPer : 1];
    // unconditional clamped loads; the correction is added and out-of-array
    // cells are zeroed when the plane is staged.  ZERO_IN: interior nodes
    // of the iterate take an offset at the end of the plane, where the
    // buffer load returns +0.0 without touching memory (the value a zeroed
    // interior holds), so only boundary nodes are read.
    auto fetch = [&](int p, double(&dst)[kIPer], float(&edst)[HAS_E ? kIPer : 1]) {
        const auto ru = plane_rsrc(uin + sxy * (size_t)p, 8u * plane_elems);
        const auto re = plane_rsrc(e32 + sxy * (size_t)p, 4u * plane_elems);
        const uint32_t skip = (ZERO_IN && p >= 1 && p <= nz - 2) ? st_int : 0u;
#pragma unroll
        for (int r = 0; r < kIPer; ++r) {
            dst[r] = bload<double>(ru, ((skip >> r) & 1) ? 8u * plane_elems : 8u * st_g[r]);
            if constexpr (HAS_E) edst[r] = bload<float>(re, 4u * st_g[r]);
        }
    };
    auto stash = [&](int p, int sl, const double(&src)[kIPer], const float(&esrc)[HAS_E ? kIPer : 1]) {
        double *dst = S + sl * SLOT;
        const bool corr = HAS_E && p >= 1 && p <= nz - 2;
#pragma unroll
        for (int r = 0; r < kIPer; ++r) {
            double v = ((st_in >> r) & 1) ? src[r] : 0.0;
            if constexpr (HAS_E) {
                if (corr && ((st_int >> r) & 1)) v += (double)esrc[r];
            }
            dst[st_l[r]] = v;
        }
    };
    double acc = 0.0;
    // planes kb-1 .. ke are read; plane p lives in register set (p - kb + 1)
    // % D and in slot (p - kb + 1) % 4.  Every step issues the same loads
    // (past the top they repeat the last plane), so the compiler waits for
    // exactly the oldest register set.
    const int pbase = kb - 1, ptop = ke;
    // planes kb .. ke-1 (at most kKZ <= 64) of cx, cy, d
    PlaneTab<double> tcx, tcy, tdd;
    tcx.load(coef, kb, 0, nz);
    tcy.load(coef, kb, 1, nz);
    tdd.load(coef, kb, 2, nz);
#pragma unroll
    for (int q = 0; q < D; ++q) {
        fetch(min(pbase + q, ptop), pre[q], epre[q]);
        __builtin_amdgcn_sched_barrier(0);
    }
    stash(pbase, 0, pre[0], epre[0]);
    stash(pbase + 1, 1, pre[1], epre[1]);
    fetch(min(pbase + D, ptop), pre[0], epre[0]);
    __builtin_amdgcn_sched_barrier(0);
    fetch(min(pbase + D + 1, ptop), pre[1], epre[1]);
    __builtin_amdgcn_sched_barrier(0);

    // step m: stage plane m+1 (into the slot of plane m-3, read two steps
    // ago), refill its register set, then the update and residual of plane
    // m (live = m < ke; a step past the top only stages and fetches)
    auto step = [&](const int m, const bool live, const int ri, const int sm, const int s0, const int sp) {
        stash(m + 1, sp, pre[ri], epre[ri]);
        fetch(min(m + 1 + D, ptop), pre[ri], epre[ri]);
        __builtin_amdgcn_sched_barrier(0);
        lds_barrier();
        if (!live) return;
        const double cx = tcx(m), cy = tcy(m), d = tdd(m);
        const double *P = S + s0 * SLOT;
        const double *Pm = S + sm * SLOT;
        const double *Pp = S + sp * SLOT;
        const auto ru = plane_rsrc(uout + sxy * (size_t)m, 8u * plane_elems);
        const auto rr = plane_rsrc(r32 + sxy * (size_t)m, 4u * plane_elems);
#pragma unroll
        for (int q = 0; q < kOwnI; ++q) {
            const int o = ow_l[q];
            const double uc = P[o];
            const double r = -(cx * (P[o + 1] + P[o - 1]) + cy * (P[o + kIWX] + P[o - kIWX]) +
                               cz * (Pp[o] + Pm[o]) + d * uc);
            if constexpr (HAS_E) bstore(uc, ru, 8u * ow_g[q]);
            bstore((float)r, rr, 4u * ow_g[q]);
            acc += ((ow_ok >> q) & 1) ? r * r : 0.0;
        }
    };
    int m0 = kb;
    for (; m0 + kRoundI <= ke; m0 += kRoundI) {
#pragma unroll
        for (int dd = 0; dd < kRoundI; ++dd)
            step(m0 + dd, true, (dd + 2) % D, dd % kSlotsI, (dd + 1) % kSlotsI, (dd + 2) % kSlotsI);
    }
    for (; m0 < ke; m0 += D) {
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            const int m = m0 + dd;
            const int t = m - kb + 1; // slot of plane m
            step(m, m < ke, (dd + 2) % D, (t + 3) % kSlotsI, t % kSlotsI, (t + 1) % kSlotsI);
        }
    }
    const double tot = block_sum<kThreads>(acc, red);
    if (tid == 0) gout<double>(it->partials)[tile - it->tile_base] = tot;
}

// ============================================================================
// Bottom solver: one workgroup runs a whole V(nu1,nu2) cycle over the small
// levels of one request, from a zero initial guess, in FP64, with exact
// red-black Gauss-Seidel ordering (a barrier between colours) and an exact
// dense solve on the coarsest grid.  Every work array lives in LDS (up to
// 160 KB on gfx950), so each phase costs LDS latency, not HBM latency.
// ============================================================================
// Threads of the bottom solver work row by row: a row is the interior nodes
// (j, k) fixed, i running; `cnt` nodes of a row go to a power-of-two group
// of 2^lg lanes and the workgroup covers 1024 / 2^lg rows at a time, so
// node coordinates come from shifts and one small division per row.
__device__ __forceinline__ int ceil_log2(int v) { return v <= 1 ? 0 : 32 - __clz(v - 1); }

template <typename Fn>
__device__ __forceinline__ void bottom_rows(int cnt, int my, int nrows, Fn &&fn)
{
    const int lg = ceil_log2(cnt);
    if ((1 << lg) > kBottomThreads) { // rows longer than the workgroup
        for (int r = 0; r < nrows; ++r) {
            const int kk = r / my;
            for (int q = (int)threadIdx.x; q < cnt; q += kBottomThreads) fn(q, r - kk * my, kk);
        }
        return;
    }
    const int q = (int)threadIdx.x & ((1 << lg) - 1);
    if (q >= cnt) return;
    for (int r = (int)threadIdx.x >> lg; r < nrows; r += kBottomThreads >> lg) {
        const int kk = r / my;
        fn(q, r - kk * my, kk);
    }
}

// One colour of red-black Gauss-Seidel on level l (colour = (i + j + k) & 1).
__device__ __forceinline__ void bottom_colour(double *smem, const BottomItem &b, int l, bool planar, int colour)
{
    const int nx = b.n[l][0], ny = b.n[l][1], nz = b.n[l][2];
    const int mx = nx - 2, my = ny - 2, mz = planar ? 1 : nz - 2;
    double *u = smem + b.off_u[l];
    const double *f = smem + b.off_f[l];
    const double *cf = smem + b.off_c[l];
    const double cz = b.cz[l];
    const int sxy = nx * ny;
    bottom_rows((mx + 1) >> 1, my, my * mz, [&](int q, int jj, int kk) {
        const int j = jj + 1, k = planar ? 0 : kk + 1;
        const int i = 1 + ((j + k + 1 + colour) & 1) + 2 * q;
        if (i > mx) return;
        const int idx = i + nx * j + sxy * k;
        double off = cf[4 * k] * (u[idx + 1] + u[idx - 1]) + cf[4 * k + 1] * (u[idx + nx] + u[idx - nx]);
        if (!planar) off += cz * (u[idx + sxy] + u[idx - sxy]);
        u[idx] = (f[idx] - off) * cf[4 * k + 3];
    });
}

__device__ __forceinline__ void bottom_smooth(double *smem, const BottomItem &b, int l, bool planar, int nsweeps)
{
    for (int s = 0; s < nsweeps; ++s) {
        bottom_colour(smem, b, l, planar, 0);
        lds_barrier();
        bottom_colour(smem, b, l, planar, 1);
        lds_barrier();
    }
}

template <typename T>
__global__ __launch_bounds__(kBottomThreads) void k_bottom(const BottomItem *__restrict__ items, int nitems)
{
    extern __shared__ double smem[];
    const BottomItem &b = items[blockIdx.x];
    if (b.state && gin<SolveState>(b.state)->done) return;
    const bool planar = b.planar != 0;
    const int tid = threadIdx.x;
    const int L = b.nlev;
    double *r = smem + b.off_r;
    // every level's u = 0 and f (the top level's from global memory), and
    // the coefficient tables, into LDS
    for (int l = 0; l < L; ++l) {
        const int N = b.n[l][0] * b.n[l][1] * b.n[l][2];
        double *u = smem + b.off_u[l];
        double *f = smem + b.off_f[l];
        const MHS_GLOBAL T *ft = gin<T>(b.f_top);
        for (int e = tid; e < N; e += kBottomThreads) {
            u[e] = 0.0;
            f[e] = (l == 0) ? (double)ft[e] : 0.0;
        }
        const int nc = 4 * b.n[l][2];
        const MHS_GLOBAL double *cg = gin<double>(b.coef[l]);
        for (int e = tid; e < nc; e += kBottomThreads) smem[b.off_c[l] + e] = cg[e];
    }
    lds_barrier();
    for (int l = 0; l < L - 1; ++l) {
        const int nx = b.n[l][0], ny = b.n[l][1], nz = b.n[l][2];
        const int sxy = nx * ny;
        const int mx = nx - 2, my = ny - 2, mz = planar ? 1 : nz - 2;
        bottom_smooth(smem, b, l, planar, b.nu1);
        // residual on interior nodes
        {
            const double *u = smem + b.off_u[l];
            const double *f = smem + b.off_f[l];
            const double *cf = smem + b.off_c[l];
            const double cz = b.cz[l];
            bottom_rows(mx, my, my * mz, [&](int q, int jj, int kk) {
                const int i = q + 1, j = jj + 1, k = planar ? 0 : kk + 1;
                const int idx = i + nx * j + sxy * k;
                double au = cf[4 * k] * (u[idx + 1] + u[idx - 1]) + cf[4 * k + 1] * (u[idx + nx] + u[idx - nx]) +
                            cf[4 * k + 2] * u[idx];
                if (!planar) au += cz * (u[idx + sxy] + u[idx - sxy]);
                r[idx] = f[idx] - au;
            });
        }
        lds_barrier();
        // full weighting onto the interior of level l+1 (within planes when
        // the step keeps z)
        {
            const int cnx = b.n[l + 1][0], cny = b.n[l + 1][1], cnz = b.n[l + 1][2];
            const bool zc = !planar && cnz < nz; // the step halves z
            const bool xyc = cnx < nx;           // the step halves x and y
            double *fc = smem + b.off_f[l + 1];
            const int cmx = cnx - 2, cmy = cny - 2, cmz = planar ? 1 : cnz - 2;
            bottom_rows(cmx, cmy, cmy * cmz, [&](int q, int jj, int kk) {
                const int I = q + 1, J = jj + 1, K = planar ? 0 : kk + 1;
                const int fidx = (xyc ? 2 * I : I) + nx * (xyc ? 2 * J : J) + sxy * (zc ? 2 * K : K);
                auto row = [&](int c) { return 0.25 * r[c - 1] + 0.5 * r[c] + 0.25 * r[c + 1]; };
                auto pl = [&](int c) { return xyc ? 0.25 * row(c - nx) + 0.5 * row(c) + 0.25 * row(c + nx) : r[c]; };
                const double v = !zc ? pl(fidx) : 0.25 * pl(fidx - sxy) + 0.5 * pl(fidx) + 0.25 * pl(fidx + sxy);
                fc[I + cnx * J + cnx * cny * K] = v;
            });
        }
        lds_barrier();
    }
    // exact solve on the coarsest grid: u = Minv f over interior nodes
    {
        const int nx = b.n[L - 1][0], ny = b.n[L - 1][1];
        const int mx = nx - 2, my = ny - 2;
        const int sxy = nx * ny;
        const int m = b.m;
        double *u = smem + b.off_u[L - 1];
        const double *f = smem + b.off_f[L - 1];
        for (int p = tid; p < m; p += kBottomThreads) {
            double acc = 0.0;
            for (int q = 0; q < m; ++q) {
                const int qi = q % mx, qr = q / mx;
                const int qj = qr % my, qk = qr / my;
                const int fidx = (qi + 1) + nx * (qj + 1) + sxy * (planar ? 0 : qk + 1);
                acc += gin<double>(b.minv)[(size_t)p * m + q] * f[fidx];
            }
            const int pi = p % mx, pr = p / mx;
            const int pj = pr % my, pk = pr / my;
            u[(pi + 1) + nx * (pj + 1) + sxy * (planar ? 0 : pk + 1)] = acc;
        }
        lds_barrier();
    }
    for (int l = L - 2; l >= 0; --l) {
        const int nx = b.n[l][0], ny = b.n[l][1], nz = b.n[l][2];
        const int cnx = b.n[l + 1][0], cny = b.n[l + 1][1];
        const bool zc = !planar && b.n[l + 1][2] < nz;
        const bool xyc = cnx < nx;
        const int sxy = nx * ny;
        const int mx = nx - 2, my = ny - 2, mz = planar ? 1 : nz - 2;
        double *u = smem + b.off_u[l];
        const double *ec = smem + b.off_u[l + 1];
        bottom_rows(mx, my, my * mz, [&](int q, int jj, int kk) {
            const int i = q + 1, j = jj + 1, k = planar ? 0 : kk + 1;
            double v;
            if (xyc) {
                v = zc ? interp3<double>(ec, cnx, cny, i, j, k)
                       : interp2<double>(ec + (size_t)cnx * cny * k, cnx, i, j);
            } else { // x and y kept: linear along z
                const double *e0 = ec + i + nx * j + sxy * (k >> 1);
                v = (k & 1) ? 0.5 * e0[0] + 0.5 * e0[sxy] : e0[0];
            }
            u[i + nx * j + sxy * k] += v;
        });
        lds_barrier();
        bottom_smooth(smem, b, l, planar, b.nu2);
    }
    {
        const int N0 = b.n[0][0] * b.n[0][1] * b.n[0][2];
        const double *u = smem + b.off_u[0];
        MHS_GLOBAL T *ut = gout<T>(b.u_top);
        for (int e = tid; e < N0; e += kBottomThreads) ut[e] = (T)u[e];
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
// (9) and (10).  A workgroup owns kTX x kFY interior nodes of `kz` planes
// (workgroups at the array edge also write the side-face nodes next to their
// tile, whose values need no differences); P planes
// are staged in LDS with a two-node halo (four planes resident, the next ones
// prefetched into a register ring) and Bz planes with a one-node halo (three
// resident).  At step m the workgroup forms Bz on plane m+1, then writes all
// five fields of plane m.  Side and top faces: B = 0.  Base plane:
// one-sided second-order z-derivatives.
// ============================================================================
constexpr int kFPX = kTX + 4;
constexpr int kFPY = kFY + 4;
constexpr int kFBX = kTX + 2;
constexpr int kFBY = kFY + 2;
constexpr int kFCells = kFPX * kFPY;
constexpr int kFPer = (kFCells + kFThreads - 1) / kFThreads;
constexpr int kDepthFields = 2; // P planes of loads in flight

__global__ __launch_bounds__(kFThreads) void k_fields(const FieldsItem *__restrict__ items, int nitems)
{
    constexpr int D = kDepthFields;
    constexpr int PSLOT = kFPY * kFPX;
    constexpr int BSLOT = kFBY * kFBX;
    constexpr int kBCells = kFBY * kFBX;
    constexpr int kBPer = (kBCells + kFThreads - 1) / kFThreads;
    constexpr int kOut = kFY * kTX / kFThreads;
    static_assert(kFY * kTX % kFThreads == 0, "whole output nodes per thread");
    __shared__ double SP[4 * PSLOT];
    __shared__ double SB[3 * BSLOT];
    const int tile = xcd_tile();
    const FieldsItem *it = items + find_item(items, nitems, tile);
    if (it->gate) {
        const auto *g = gin<SolveState>(it->gate);
        const int cycles = g->checks - 1;
        if (g->done != kConverged || cycles < it->gate_min || (it->gate_odd >= 0 && (cycles & 1) != it->gate_odd))
            return;
    }
    const MHS_GLOBAL double *__restrict__ P = gin<double>(it->P);
    const int nx = it->nx, ny = it->ny, nz = it->nz;
    const int kz = it->kz;
    int local = tile - it->tile_base;
    const int tx = local % it->ntx;
    local /= it->ntx;
    const int ty = local % it->nty;
    const int tz = local / it->nty;
    const int i0 = 1 + tx * kTX, j0 = 1 + ty * kFY;
    const int kb = tz * kz;
    const int ke = min(kb + kz, nz);
    const size_t sxy = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const double ix2 = 1.0 / (it->dx * it->dx), iy2 = 1.0 / (it->dy * it->dy);
    const double i2dx = 0.5 / it->dx, i2dy = 0.5 / it->dy, i2dz = 0.5 / it->dz;
    const double alpha = it->alpha, mu0 = it->mu0, g = it->g;
    const MHS_CONST double *tab = gconst<double>(it->tab);
    MHS_GLOBAL double *__restrict__ oBx = gout<double>(it->Bx);
    MHS_GLOBAL double *__restrict__ oBy = gout<double>(it->By);
    MHS_GLOBAL double *__restrict__ oBz = gout<double>(it->Bz);
    MHS_GLOBAL double *__restrict__ op = gout<double>(it->p);
    MHS_GLOBAL double *__restrict__ orho = gout<double>(it->rho);

    // ---- per-thread geometry, fixed for the whole z-march ------------------
    // P window cells staged (two-node halo)
    int st_l[kFPer];
    uint32_t st_g[kFPer];
    uint32_t st_in = 0;
#pragma unroll
    for (int r = 0; r < kFPer; ++r) {
        const int e = tid + r * kFThreads;
        const int ee = min(e, kFCells - 1);
        const int w = ee / kFPX, c = ee - w * kFPX;
        const int i = i0 - 2 + c, j = j0 - 2 + w;
        st_l[r] = e < kFCells ? ee : -1;
        st_g[r] = (uint32_t)(min(max(i, 0), nx - 1) + nx * min(max(j, 0), ny - 1));
        if (i >= 0 && i < nx && j >= 0 && j < ny) st_in |= 1u << r;
    }
    // Bz cells formed (one-node halo): SB index and SP centre; interior flag
    uint32_t bz_i[kBPer];
    uint32_t bz_int = 0;
#pragma unroll
    for (int r = 0; r < kBPer; ++r) {
        const int e = tid + r * kFThreads;
        const int ee = min(e, kBCells - 1);
        const int w = ee / kFBX, c = ee - w * kFBX;
        const int i = i0 - 1 + c, j = j0 - 1 + w;
        bz_i[r] = pk16(e < kBCells ? ee : kNone, (w + 1) * kFPX + (c + 1));
        if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) bz_int |= 1u << r;
    }
    // output nodes: nodes past the interior are redirected to the nearest
    // interior node, which they recompute identically, so every lane stores
    uint32_t o_i[kOut];
    uint32_t o_g[kOut];
    uint32_t o_int = 0;
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
        const int e = tid + q * kFThreads;
        const int i = min(i0 + e % kTX, nx - 2), j = min(j0 + e / kTX, ny - 2);
        const int w = j - j0, c = i - i0;
        o_i[q] = pk16((w + 2) * kFPX + (c + 2), (w + 1) * kFBX + (c + 1));
        o_g[q] = (uint32_t)(i + nx * j);
        if (i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2) o_int |= 1u << q;
    }
    // side-face nodes next to the tile (at most one per thread): the x faces
    // over the tile's rows extended to the y faces, then the y faces over the
    // tile's columns.  B = 0 there, so p = p_b and rho = rho_b.
    static_assert(2 * (kFY + 2) + 2 * kTX <= kFThreads, "one face node per thread");
    uint32_t f_g = 0;
    bool f_ok = false;
    {
        const bool xlo = tx == 0, xhi = tx == it->ntx - 1, ylo = ty == 0, yhi = ty == it->nty - 1;
        const int jb = ylo ? 0 : j0, je = yhi ? ny - 1 : j0 + kFY - 1; // rows of the x faces
        const int ie = min(i0 + kTX - 1, nx - 2);                      // last interior column
        const int nxf = je - jb + 1, nyf = ie - i0 + 1;
        int e = tid, fi = -1, fj = -1;
        if (xlo) {
            if (e < nxf) fi = 0, fj = jb + e;
            e -= nxf;
        }
        if (xhi && fi < 0) {
            if (e >= 0 && e < nxf) fi = nx - 1, fj = jb + e;
            e -= nxf;
        }
        if (ylo && fi < 0) {
            if (e >= 0 && e < nyf) fi = i0 + e, fj = 0;
            e -= nyf;
        }
        if (yhi && fi < 0) {
            if (e >= 0 && e < nyf) fi = i0 + e, fj = ny - 1;
        }
        if (fi >= 0) {
            f_ok = true;
            f_g = (uint32_t)(fi + nx * fj);
        }
    }

    double pre[D][kFPer];
    // unconditional clamped loads; out-of-array cells zeroed when staged
    auto fetch = [&](int p, double(&dst)[kFPer]) {
        const MHS_GLOBAL double *pl = P + sxy * (size_t)min(p, nz - 1);
#pragma unroll
        for (int r = 0; r < kFPer; ++r) dst[r] = pl[st_g[r]];
    };
    auto stash = [&](int p, const double(&src)[kFPer]) {
        double *dst = SP + (p & 3) * PSLOT;
#pragma unroll
        for (int r = 0; r < kFPer; ++r)
            if (st_l[r] >= 0) dst[st_l[r]] = ((st_in >> r) & 1) ? src[r] : 0.0;
    };
    // Bz = -(d2x + d2y) P on plane p, one-node ring; 0 on faces and the top
    auto bz_plane = [&](int p) {
        const double *src = SP + (p & 3) * PSLOT;
        double *dst = SB + (p % 3) * BSLOT;
        const bool plane_ok = p <= nz - 2;
#pragma unroll
        for (int r = 0; r < kBPer; ++r) {
            const int l = lo16(bz_i[r]);
            if (l == kNone) continue;
            const int s = hi16(bz_i[r]);
            double v = 0.0;
            if (plane_ok && ((bz_int >> r) & 1))
                v = -((src[s + 1] - 2.0 * src[s] + src[s - 1]) * ix2 + (src[s + kFPX] - 2.0 * src[s] + src[s - kFPX]) * iy2);
            dst[l] = v;
        }
    };

    // P planes q0 .. q0+2 staged and Bz q0 .. q0+1 formed up front (the
    // base plane also needs Bz on plane 2); then step m forms Bz(m+1),
    // writes plane m and stages P(m+2) from the register ring, which runs D
    // planes ahead.
    const int q0 = (kb == 0) ? 0 : kb - 1;
    {
        double tmp[kFPer];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            fetch(q0 + q, tmp);
            stash(q0 + q, tmp);
        }
    }
    // register set d holds plane kb + 2 + d (+ D per round); every step
    // refills its set unconditionally (past the top it repeats the last
    // plane), so the compiler can wait for exactly the oldest set
#pragma unroll
    for (int q = 0; q < D; ++q) {
        fetch(kb + 2 + q, pre[q]);
        __builtin_amdgcn_sched_barrier(0);
    }
    lds_barrier();
    bz_plane(q0);
    bz_plane(q0 + 1);
    if (kb == 0) bz_plane(2);
    for (int m0 = kb; m0 < ke; m0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int m = m0 + d;
            if (m >= ke) break;
            if (m + 1 >= (kb == 0 ? 3 : q0 + 2)) bz_plane(min(m + 1, nz - 1));
            lds_barrier();
            const double xi = tab[m], dxi = tab[nz + m], pb = tab[2 * nz + m], rhob = tab[3 * nz + m];
            const double *Pc = SP + (m & 3) * PSLOT;
            const double *Bc = SB + (m % 3) * BSLOT;
            const bool plane_ok = m <= nz - 2;
#pragma unroll
            for (int q = 0; q < kOut; ++q) {
                double bx = 0.0, by = 0.0, bz = 0.0, p = pb, rho = rhob;
                if (plane_ok && ((o_int >> q) & 1)) {
                    const int pc = lo16(o_i[q]), bc = hi16(o_i[q]);
                    double dzp_xp, dzp_xm, dzp_yp, dzp_ym, dbzz;
                    if (m >= 1) {
                        const double *Pu = SP + ((m + 1) & 3) * PSLOT;
                        const double *Pd = SP + ((m - 1) & 3) * PSLOT;
                        dzp_xp = (Pu[pc + 1] - Pd[pc + 1]) * i2dz;
                        dzp_xm = (Pu[pc - 1] - Pd[pc - 1]) * i2dz;
                        dzp_yp = (Pu[pc + kFPX] - Pd[pc + kFPX]) * i2dz;
                        dzp_ym = (Pu[pc - kFPX] - Pd[pc - kFPX]) * i2dz;
                        dbzz = (SB[((m + 1) % 3) * BSLOT + bc] - SB[((m + 2) % 3) * BSLOT + bc]) * i2dz;
                    } else {
                        const double *P1 = SP + PSLOT;
                        const double *P2 = SP + 2 * PSLOT;
                        auto one = [&](int a) { return (-3.0 * Pc[a] + 4.0 * P1[a] - P2[a]) * i2dz; };
                        dzp_xp = one(pc + 1);
                        dzp_xm = one(pc - 1);
                        dzp_yp = one(pc + kFPX);
                        dzp_ym = one(pc - kFPX);
                        dbzz = (-3.0 * SB[bc] + 4.0 * SB[BSLOT + bc] - SB[2 * BSLOT + bc]) * i2dz;
                    }
                    bx = alpha * (Pc[pc + kFPX] - Pc[pc - kFPX]) * i2dy + (dzp_xp - dzp_xm) * i2dx;
                    by = -alpha * (Pc[pc + 1] - Pc[pc - 1]) * i2dx + (dzp_yp - dzp_ym) * i2dy;
                    bz = Bc[bc];
                    const double dbzx = (Bc[bc + 1] - Bc[bc - 1]) * i2dx;
                    const double dbzy = (Bc[bc + kFBX] - Bc[bc - kFBX]) * i2dy;
                    const double bz2 = bz * bz;
                    p = pb - xi * bz2 / (2.0 * mu0);
                    rho = rhob + (dxi * bz2 / (2.0 * mu0) + xi * (bx * dbzx + by * dbzy + bz * dbzz) / mu0) / g;
                }
                const size_t idx = (size_t)o_g[q] + sxy * (size_t)m;
                oBx[idx] = bx;
                oBy[idx] = by;
                oBz[idx] = bz;
                op[idx] = p;
                orho[idx] = rho;
            }
            if (f_ok) {
                const size_t idx = (size_t)f_g + sxy * (size_t)m;
                oBx[idx] = 0.0;
                oBy[idx] = 0.0;
                oBz[idx] = 0.0;
                op[idx] = pb;
                orho[idx] = rhob;
            }
            // P(m+2) replaces the slot of plane m-2, last read a step ago
            if (m + 2 >= q0 + 3) stash(m + 2, pre[d]);
            fetch(m + 2 + D, pre[d]);
            lds_barrier();
        }
    }
}

// ============================================================================
// Diagnostics of equations (1)-(3): j = curl B / mu0, the force-balance
// residual |j x B - grad p - rho g e_z| and div B, by the differences of the
// field recovery (central; one-sided second order at the base plane), zero on
// the side and top faces.  One thread per (x, y) column marches a chunk of
// planes; the values it needs on plane k+1 (its column of Bx, By, Bz, p and
// their in-plane neighbours, rho) are loaded while plane k is computed.
// In-plane neighbours come from the caches (the kernel is a diagnostic, off
// the solve's path).  Contraction is off so that every value is rounded as
// the differences are written (the oracle evaluates the same expressions).
// ============================================================================
constexpr int kDX = 64, kDY = 4;
static_assert(kDX * kDY == kThreads, "diagnostics tile is one workgroup");

__global__ __launch_bounds__(kThreads) void k_diag(const DiagItem it)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kDX + (int)(threadIdx.x % kDX);
    const int j = blockIdx.y * kDY + (int)(threadIdx.x / kDX);
    const int nx = it.nx, ny = it.ny, nz = it.nz;
    if (i >= nx || j >= ny) return;
    const int k0 = blockIdx.z * it.kz;
    const int k1 = min(k0 + it.kz, nz);
    const size_t sxy = (size_t)nx * ny;
    const size_t col = (size_t)i + (size_t)nx * j;
    const bool side = i == 0 || i == nx - 1 || j == 0 || j == ny - 1;
    const MHS_GLOBAL double *Bx = gin<double>(it.Bx), *By = gin<double>(it.By), *Bz = gin<double>(it.Bz);
    const MHS_GLOBAL double *pp = gin<double>(it.p), *rho = gin<double>(it.rho);
    MHS_GLOBAL double *ojx = gout<double>(it.jx), *ojy = gout<double>(it.jy), *ojz = gout<double>(it.jz);
    MHS_GLOBAL double *ofr = gout<double>(it.fres), *odv = gout<double>(it.divb);
    const double tdx = 2.0 * it.dx, tdy = 2.0 * it.dy, tdz = 2.0 * it.dz;
    // in-plane neighbour offsets (clamped: side columns write zeros anyway)
    const size_t xm = col - (i > 0 ? 1 : 0), xp = col + (i < nx - 1 ? 1 : 0);
    const size_t ym = col - (j > 0 ? (size_t)nx : 0), yp = col + (j < ny - 1 ? (size_t)nx : 0);
    struct Col {
        double bx, by, bz, p;
    };
    // in-plane neighbours of the column on one plane, and rho there
    struct Nb {
        double bx_xp, bx_xm, bx_yp, bx_ym, by_xp, by_xm, by_yp, by_ym;
        double bz_xp, bz_xm, bz_yp, bz_ym, p_xp, p_xm, p_yp, p_ym, rho;
    };
    // byte offsets within a plane; loads go through per-plane buffer
    // resources, so the per-lane address state is these five words
    const uint32_t bc = 8u * (uint32_t)col, bxp = 8u * (uint32_t)xp, bxm = 8u * (uint32_t)xm;
    const uint32_t byp = 8u * (uint32_t)yp, bym = 8u * (uint32_t)ym;
    const uint32_t plane_bytes = 8u * (uint32_t)sxy;
    auto load_col = [&](int k) {
        const size_t pl = sxy * (size_t)min(max(k, 0), nz - 1);
        return Col{bload<double>(plane_rsrc(Bx + pl, plane_bytes), bc), bload<double>(plane_rsrc(By + pl, plane_bytes), bc),
                   bload<double>(plane_rsrc(Bz + pl, plane_bytes), bc), bload<double>(plane_rsrc(pp + pl, plane_bytes), bc)};
    };
    auto load_nb = [&](int k) {
        const size_t pl = sxy * (size_t)min(max(k, 0), nz - 1);
        const auto rx = plane_rsrc(Bx + pl, plane_bytes), ry = plane_rsrc(By + pl, plane_bytes);
        const auto rz = plane_rsrc(Bz + pl, plane_bytes), rp = plane_rsrc(pp + pl, plane_bytes);
        Nb q;
        q.bx_xp = bload<double>(rx, bxp), q.bx_xm = bload<double>(rx, bxm);
        q.bx_yp = bload<double>(rx, byp), q.bx_ym = bload<double>(rx, bym);
        q.by_xp = bload<double>(ry, bxp), q.by_xm = bload<double>(ry, bxm);
        q.by_yp = bload<double>(ry, byp), q.by_ym = bload<double>(ry, bym);
        q.bz_xp = bload<double>(rz, bxp), q.bz_xm = bload<double>(rz, bxm);
        q.bz_yp = bload<double>(rz, byp), q.bz_ym = bload<double>(rz, bym);
        q.p_xp = bload<double>(rp, bxp), q.p_xm = bload<double>(rp, bxm);
        q.p_yp = bload<double>(rp, byp), q.p_ym = bload<double>(rp, bym);
        q.rho = bload<double>(plane_rsrc(rho + pl, plane_bytes), bc);
        return q;
    };
    // columns k-1, k, k+1 and the neighbours of plane k in hand; each step
    // issues the loads of column k+2 and of plane k+1's neighbours first
    Col m = load_col(k0 - 1), c = load_col(k0), u = load_col(k0 + 1);
    Nb nb = load_nb(k0);
    for (int k = k0; k < k1; ++k) {
        const Col u2 = load_col(k + 2);
        const Nb nbn = load_nb(k + 1);
        const Col w = k == 0 ? u2 : u; // plane 2 for the one-sided base difference
        double jx = 0.0, jy = 0.0, jz = 0.0, fr = 0.0, dv = 0.0;
        if (!side && k < nz - 1) {
            const Nb &q = nb;
            // z-derivatives: central, or one-sided at the base
            double dzbx, dzby, dzbz, dzp;
            if (k > 0) {
                dzbx = (u.bx - m.bx) / tdz;
                dzby = (u.by - m.by) / tdz;
                dzbz = (u.bz - m.bz) / tdz;
                dzp = (u.p - m.p) / tdz;
            } else {
                dzbx = (-3.0 * c.bx + 4.0 * u.bx - w.bx) / tdz;
                dzby = (-3.0 * c.by + 4.0 * u.by - w.by) / tdz;
                dzbz = (-3.0 * c.bz + 4.0 * u.bz - w.bz) / tdz;
                dzp = (-3.0 * c.p + 4.0 * u.p - w.p) / tdz;
            }
            const double dxbx = (q.bx_xp - q.bx_xm) / tdx, dybx = (q.bx_yp - q.bx_ym) / tdy;
            const double dxby = (q.by_xp - q.by_xm) / tdx, dyby = (q.by_yp - q.by_ym) / tdy;
            const double dxbz = (q.bz_xp - q.bz_xm) / tdx, dybz = (q.bz_yp - q.bz_ym) / tdy;
            const double dxp = (q.p_xp - q.p_xm) / tdx, dyp = (q.p_yp - q.p_ym) / tdy;
            jx = (dybz - dzby) / it.mu0;
            jy = (dzbx - dxbz) / it.mu0;
            jz = (dxby - dybx) / it.mu0;
            const double fx = (jy * c.bz - jz * c.by) - dxp;
            const double fy = (jz * c.bx - jx * c.bz) - dyp;
            const double fz = (jx * c.by - jy * c.bx) - dzp - q.rho * it.g;
            fr = sqrt(fx * fx + fy * fy + fz * fz);
            dv = dxbx + dyby + dzbz;
        }
        const size_t pl = sxy * (size_t)k;
        bstore(jx, plane_rsrc(ojx + pl, plane_bytes), bc);
        bstore(jy, plane_rsrc(ojy + pl, plane_bytes), bc);
        bstore(jz, plane_rsrc(ojz + pl, plane_bytes), bc);
        bstore(fr, plane_rsrc(ofr + pl, plane_bytes), bc);
        bstore(dv, plane_rsrc(odv + pl, plane_bytes), bc);
        m = c;
        c = u;
        u = u2;
        nb = nbn;
    }
}

// ============================================================================
// Field lines (the curves of Section 3's figures): dx/ds = B/|B| in arc
// length, classical fourth-order Runge-Kutta with a fixed step ds, B between
// nodes by trilinear interpolation (nested linear interpolations a + t (b -
// a) along x, then y, then z, coordinates clamped to the box).  A line ends
// when a step would leave the box (kTraceExit; that point is not written),
// when a stage finds |B| <= bmin (kTraceNull), or after max_steps steps.
// One thread per line; point n of line l is at points[3 (n nlines + l)], so
// the lanes of a wave write consecutive records.  Contraction is off: every
// operation is rounded as written, as in the oracle's definition.
// ============================================================================
constexpr int kTraceThreads = 256;
enum TraceStatus : int32_t { kTraceMaxSteps = 0, kTraceExit = 1, kTraceNull = 2 };

__global__ __launch_bounds__(kTraceThreads) void k_trace(const TraceItem it)
{
#pragma clang fp contract(off)
    const int l = blockIdx.x * kTraceThreads + (int)threadIdx.x;
    if (l >= it.nlines) return;
    const MHS_GLOBAL double *Bx = gin<double>(it.Bx), *By = gin<double>(it.By), *Bz = gin<double>(it.Bz);
    const MHS_GLOBAL double *seed = gin<double>(it.seeds) + 3 * (size_t)l;
    MHS_GLOBAL double *pts = gout<double>(it.points);
    const size_t rec = 3 * (size_t)it.nlines; // doubles per step
    const int nx = it.nx, ny = it.ny;
    const size_t sxy = (size_t)nx * ny;
    auto locate = [](double x, double len, double h, int n, int &i, double &t) {
        const double p = fmin(fmax(x, 0.0), len);
        const double f = p / h;
        i = min((int)floor(f), n - 2);
        t = f - (double)i;
    };
    auto lerp = [](double a, double b, double t) { return a + t * (b - a); };
    // unit tangent at (x, y, z); false when |B| <= bmin
    auto tangent = [&](double x, double y, double z, double &tx, double &ty, double &tz) {
        int i, j, k;
        double fx, fy, fz;
        locate(x, it.lx, it.dx, nx, i, fx);
        locate(y, it.ly, it.dy, ny, j, fy);
        locate(z, it.lz, it.dz, it.nz, k, fz);
        const size_t c = (size_t)i + (size_t)nx * j + sxy * k;
        auto trilin = [&](const MHS_GLOBAL double *F) {
            const double c00 = lerp(F[c], F[c + 1], fx);
            const double c10 = lerp(F[c + nx], F[c + nx + 1], fx);
            const double c01 = lerp(F[c + sxy], F[c + sxy + 1], fx);
            const double c11 = lerp(F[c + sxy + nx], F[c + sxy + nx + 1], fx);
            return lerp(lerp(c00, c10, fy), lerp(c01, c11, fy), fz);
        };
        const double bx = trilin(Bx), by = trilin(By), bz = trilin(Bz);
        const double b = sqrt((bx * bx + by * by) + bz * bz);
        if (!(b > it.bmin)) return false;
        tx = bx / b;
        ty = by / b;
        tz = bz / b;
        return true;
    };
    auto inside = [&](double x, double y, double z) {
        return x >= 0.0 && x <= it.lx && y >= 0.0 && y <= it.ly && z >= 0.0 && z <= it.lz;
    };
    double x = seed[0], y = seed[1], z = seed[2];
    MHS_GLOBAL double *o = pts + 3 * (size_t)l;
    o[0] = x;
    o[1] = y;
    o[2] = z;
    const double ds = it.ds, hh = 0.5 * ds, h6 = ds / 6.0;
    int n = 0;
    int32_t st = kTraceMaxSteps;
    if (!inside(x, y, z)) {
        st = kTraceExit;
    } else {
        for (; n < it.max_steps; ++n) {
            double k1x, k1y, k1z, k2x, k2y, k2z, k3x, k3y, k3z, k4x, k4y, k4z;
            if (!tangent(x, y, z, k1x, k1y, k1z) ||
                !tangent(x + hh * k1x, y + hh * k1y, z + hh * k1z, k2x, k2y, k2z) ||
                !tangent(x + hh * k2x, y + hh * k2y, z + hh * k2z, k3x, k3y, k3z) ||
                !tangent(x + ds * k3x, y + ds * k3y, z + ds * k3z, k4x, k4y, k4z)) {
                st = kTraceNull;
                break;
            }
            const double qx = x + h6 * (((k1x + 2.0 * k2x) + 2.0 * k3x) + k4x);
            const double qy = y + h6 * (((k1y + 2.0 * k2y) + 2.0 * k3y) + k4y);
            const double qz = z + h6 * (((k1z + 2.0 * k2z) + 2.0 * k3z) + k4z);
            if (!inside(qx, qy, qz)) {
                st = kTraceExit;
                break;
            }
            x = qx;
            y = qy;
            z = qz;
            o += rec;
            o[0] = x;
            o[1] = y;
            o[2] = z;
        }
    }
    gout<int32_t>(it.count)[l] = n + 1;
    gout<int32_t>(it.status)[l] = st;
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
// the twin's faces equal P's faces.  With `swap` (cold starts only) the
// solve starts from the twin: its interior is zeroed and P's is not touched.
// With `keep` no interior is written: the refinement steps that read the
// start iterate take its interior as zero.
__global__ __launch_bounds__(256) void k_prep3(const PrepItem *__restrict__ items, int nitems)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const PrepItem &it = items[find_prep(items, nitems, g)];
    const int64_t e0 = (g - it.base) * kPrepNodes;
    if (e0 >= it.n) return;
    const int nx = it.nx, ny = it.ny, nz = it.nz;
    if (it.keep) {
        // only the boundary nodes: planes 0 and nz - 1, then the ring of
        // every plane between (rows j = 0 and ny - 1, columns i = 0 and
        // nx - 1); it.n counts them
        const uint32_t pl = (uint32_t)nx * (uint32_t)ny, ring = 2u * (uint32_t)nx + 2u * (uint32_t)(ny - 2);
#pragma unroll
        for (int q = 0; q < kPrepNodes; ++q) {
            const int64_t fq = e0 + q;
            if (fq >= it.n) break;
            const uint32_t f = (uint32_t)fq;
            int i, j, k;
            if (f < 2u * pl) {
                const uint32_t a = f < pl ? f : f - pl;
                k = f < pl ? 0 : nz - 1;
                j = (int)(a / (uint32_t)nx);
                i = (int)(a - (uint32_t)j * (uint32_t)nx);
            } else {
                const uint32_t b = f - 2u * pl, kk = b / ring, r = b - kk * ring;
                k = 1 + (int)kk;
                if (r < 2u * (uint32_t)nx) {
                    j = r < (uint32_t)nx ? 0 : ny - 1;
                    i = (int)(r < (uint32_t)nx ? r : r - (uint32_t)nx);
                } else {
                    const uint32_t c = r - 2u * (uint32_t)nx;
                    i = c < (uint32_t)(ny - 2) ? 0 : nx - 1;
                    j = 1 + (int)(c < (uint32_t)(ny - 2) ? c : c - (uint32_t)(ny - 2));
                }
            }
            const int64_t e = (int64_t)i + (int64_t)nx * ((int64_t)j + (int64_t)ny * k);
            const bool side = (i == 0 || i == nx - 1 || j == 0 || j == ny - 1);
            if (k == 0) {
                if (side && !it.faces) it.P[e] = 0.0;
                if (it.twin) it.twin[e] = (side && !it.faces) ? 0.0 : it.P[e];
            } else {
                if (!it.faces) it.P[e] = 0.0;
                if (it.twin) it.twin[e] = it.faces ? it.P[e] : 0.0;
            }
        }
        return;
    }
    // kPrepNodes consecutive nodes per thread: the divisions for the first,
    // then stepping along x (32-bit index arithmetic: a plan's grids have
    // fewer than 2^31 nodes)
    const uint32_t e32 = (uint32_t)e0, r = e32 / (uint32_t)nx;
    int i = (int)(e32 - r * (uint32_t)nx);
    const uint32_t kk = r / (uint32_t)ny;
    int j = (int)(r - kk * (uint32_t)ny), k = (int)kk;
#pragma unroll
    for (int q = 0; q < kPrepNodes; ++q) {
        const int64_t e = e0 + q;
        if (e >= it.n) break;
        const bool side = (i == 0 || i == nx - 1 || j == 0 || j == ny - 1);
        if (k == 0) {
            if (side && !it.faces) it.P[e] = 0.0;
            if (it.twin) it.twin[e] = (side && !it.faces) ? 0.0 : it.P[e];
        } else if (side || k == nz - 1) {
            if (!it.faces) it.P[e] = 0.0;
            if (it.twin) it.twin[e] = it.faces ? it.P[e] : 0.0;
        } else if (it.swap) {
            it.twin[e] = 0.0;
        } else if (!it.warm) {
            it.P[e] = 0.0;
        }
        if (++i == nx) {
            i = 0;
            if (++j == ny) {
                j = 0;
                ++k;
            }
        }
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
    if (edge ? !it.faces : !it.warm) it.P[e] = 0.0;
    if (edge && it.twin) it.twin[e] = it.faces ? it.P[e] : 0.0;
}

// dst = src; skipped once `skip` (if given) reports a finished solve.
__global__ __launch_bounds__(256) void k_copy(const double *__restrict__ src, double *__restrict__ dst, int64_t n,
                                              const SolveState *skip)
{
    if (skip && skip->done) return;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = src[e];
}

// dst[0 .. n) = 0 in 16-byte words (a fill kernel rather than a memset, so
// the clear can sit in a captured stream).
__global__ __launch_bounds__(256) void k_zero(uint4 *__restrict__ dst, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
        dst[e] = make_uint4(0u, 0u, 0u, 0u);
}

template <typename T>
hipError_t sweep3_dispatch(const LevelItem *items, int nitems, int ntiles, int flags, hipStream_t s)
{
    dim3 grid(ntiles), block(kSThreads);
    switch (flags & 15) {
#define MHS_CASE(F)                                                                      \
    case F:                                                                              \
        hipLaunchKernelGGL((k_sweep3<T, F>), grid, block, 0, s, items, nitems);         \
        break;
        // the variants the cycle builders and stage entry points launch:
        // plain, with f, first sweep from zero, with the norm of the input,
        // with the prolongation (other combinations never occur)
        MHS_CASE(0) MHS_CASE(1) MHS_CASE(3) MHS_CASE(4) MHS_CASE(5) MHS_CASE(8) MHS_CASE(9)
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
    switch (flags & 31) {
#define MHS_CASE(F)                                                                      \
    case F:                                                                              \
        hipLaunchKernelGGL((k_sweep2<T, F>), grid, block, 0, s, items, nitems);         \
        break;
        // the variants the cycle builders and stage entry points launch:
        // plain, with f, first sweep from zero, with the norm of the input,
        // with the prolongation (other combinations never occur), each as
        // one sweep or two
        MHS_CASE(0) MHS_CASE(1) MHS_CASE(3) MHS_CASE(4) MHS_CASE(5) MHS_CASE(8) MHS_CASE(9)
        MHS_CASE(16) MHS_CASE(17) MHS_CASE(19) MHS_CASE(20) MHS_CASE(21) MHS_CASE(24) MHS_CASE(25)
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

template <typename T, bool HAS_F>
static void restrict3_variant(const LevelItem *items, int nitems, dim3 grid, bool keepz, hipStream_t s)
{
    if (keepz)
        hipLaunchKernelGGL((k_restrict3<T, HAS_F, true>), grid, dim3(kThreads), 0, s, items, nitems);
    else
        hipLaunchKernelGGL((k_restrict3<T, HAS_F, false>), grid, dim3(kThreads), 0, s, items, nitems);
}

hipError_t launch_restrict3(const LevelItem *items, int nitems, int ntiles, bool has_f, bool keepz, bool dbl,
                            hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles);
    if (dbl) {
        if (has_f)
            restrict3_variant<double, true>(items, nitems, grid, keepz, s);
        else
            restrict3_variant<double, false>(items, nitems, grid, keepz, s);
    } else {
        if (has_f)
            restrict3_variant<float, true>(items, nitems, grid, keepz, s);
        else
            restrict3_variant<float, false>(items, nitems, grid, keepz, s);
    }
    return hipGetLastError();
}

hipError_t launch_restrict3_z(const LevelItem *items, int nitems, int ntiles, bool has_f, bool dbl, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(kThreads);
    if (dbl) {
        if (has_f)
            hipLaunchKernelGGL((k_restrict3_z<double, true>), grid, block, 0, s, items, nitems);
        else
            hipLaunchKernelGGL((k_restrict3_z<double, false>), grid, block, 0, s, items, nitems);
    } else {
        if (has_f)
            hipLaunchKernelGGL((k_restrict3_z<float, true>), grid, block, 0, s, items, nitems);
        else
            hipLaunchKernelGGL((k_restrict3_z<float, false>), grid, block, 0, s, items, nitems);
    }
    return hipGetLastError();
}

hipError_t launch_prolong3_z(const LevelItem *items, int nitems, int ntiles, bool dbl, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(kThreads);
    if (dbl)
        hipLaunchKernelGGL((k_prolong3_z<double>), grid, block, 0, s, items, nitems);
    else
        hipLaunchKernelGGL((k_prolong3_z<float>), grid, block, 0, s, items, nitems);
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

hipError_t launch_ir3(const LevelItem *items, int nitems, int ntiles, bool has_e, bool zero_in, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(kThreads);
    if (has_e && zero_in)
        hipLaunchKernelGGL((k_ir3<true, true>), grid, block, 0, s, items, nitems);
    else if (has_e)
        hipLaunchKernelGGL((k_ir3<true, false>), grid, block, 0, s, items, nitems);
    else if (zero_in)
        hipLaunchKernelGGL((k_ir3<false, true>), grid, block, 0, s, items, nitems);
    else
        hipLaunchKernelGGL((k_ir3<false, false>), grid, block, 0, s, items, nitems);
    return hipGetLastError();
}

hipError_t launch_bottom(const BottomItem *items, int nitems, int lds_bytes, bool dbl, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (lds_bytes <= 0 || lds_bytes > kBottomLdsMax) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bottom<double>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kBottomLdsMax);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bottom<float>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kBottomLdsMax);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    dim3 grid(nitems), block(kBottomThreads);
    if (dbl)
        hipLaunchKernelGGL((k_bottom<double>), grid, block, lds_bytes, s, items, nitems);
    else
        hipLaunchKernelGGL((k_bottom<float>), grid, block, lds_bytes, s, items, nitems);
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
    hipLaunchKernelGGL(k_fields, dim3(ntiles), dim3(kFThreads), 0, s, items, nitems);
    return hipGetLastError();
}

hipError_t launch_diag(const DiagItem &item, hipStream_t s)
{
    const dim3 grid((unsigned)((item.nx + kDX - 1) / kDX), (unsigned)((item.ny + kDY - 1) / kDY),
                    (unsigned)((item.nz + item.kz - 1) / item.kz));
    hipLaunchKernelGGL(k_diag, grid, dim3(kThreads), 0, s, item);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceItem &item, hipStream_t s)
{
    if (item.nlines <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((item.nlines + kTraceThreads - 1) / kTraceThreads);
    hipLaunchKernelGGL(k_trace, dim3(blocks), dim3(kTraceThreads), 0, s, item);
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

hipError_t launch_zero(void *dst, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    if (((uintptr_t)dst | bytes) & 15) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 16);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint4 *)dst, n);
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
