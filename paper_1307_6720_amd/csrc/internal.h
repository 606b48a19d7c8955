// Internal declarations shared by the host library and the kernels.
//
// Every kernel is descriptor-driven: it receives a device array of work
// items (one per request/level it serves) and maps its workgroups onto the
// items' tiles through a prefix of tile counts.  A single solve launches
// one item per stage; the batched (serving) path launches many.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mhs {

constexpr int kMaxLevels = 16;

// ---- tile geometry ---------------------------------------------------------
// 3D refinement residual: x-y tile of kTX x kTY interior nodes, marching
// kKZ planes in z; 256 threads (the smoother's tile height is kSTY below).
#ifndef MHS_TILE_Y
#define MHS_TILE_Y 8
#endif
#ifndef MHS_RING_DEPTH_F
#define MHS_RING_DEPTH_F 2
#endif
// The 3D smoother is unrolled over ten steps; without a bound the register
// allocator may take more than 128 VGPRs and drop below four workgroups per
// compute unit, which the level-0 launch (four workgroups per CU) needs.
#ifndef MHS_SWEEP_ATTR
#define MHS_SWEEP_ATTR __attribute__((amdgpu_waves_per_eu(4)))
#endif
#ifndef MHS_SWEEP_HP32
#define MHS_SWEEP_HP32 48
#endif
#ifndef MHS_SWEEP_RW32
#define MHS_SWEEP_RW32 98
#endif
#ifndef MHS_SWEEP_ROWMAP32
#define MHS_SWEEP_ROWMAP32 1
#endif
#ifndef MHS_SWEEP_HP64
#define MHS_SWEEP_HP64 40
#endif
#ifndef MHS_RING_DEPTH
#define MHS_RING_DEPTH 2
#endif
constexpr int kTX = 64;
constexpr int kTY = MHS_TILE_Y;
constexpr int kKZ = 32;
constexpr int kThreads = 256;
// The 3D smoother's own tile height: one black node of the tile per thread,
// so a workgroup of kSTY * kTX / 2 threads.  Taller tiles stage fewer halo
// cells per updated node and recompute fewer red nodes of the ring.
#ifndef MHS_SWEEP_TILE_Y
#define MHS_SWEEP_TILE_Y 16
#endif
constexpr int kSTY = MHS_SWEEP_TILE_Y;
constexpr int kSThreads = kSTY * kTX / 2;
static_assert(kSThreads % 64 == 0 && kSThreads <= 1024, "smoother workgroup size");
// planes of HBM loads a marching kernel keeps in flight (register ring)
constexpr int kDepth = MHS_RING_DEPTH;
constexpr int kDepthF = MHS_RING_DEPTH_F; // with right-hand side or prolongation
// 3D residual + restriction: kCX x kCY coarse nodes per workgroup, marching
// kKC coarse planes.
constexpr int kCX = 32;
constexpr int kCY = 8;
constexpr int kKC = 16;
// 2D smoother: kTX x kTY2 interior nodes per workgroup.
constexpr int kTY2 = 16;
// field recovery: kTX x kFY nodes per workgroup of kFThreads threads (four
// nodes per thread), marching kKZ planes.
#ifndef MHS_FIELDS_TILE_Y
#define MHS_FIELDS_TILE_Y 16
#endif
#ifndef MHS_FIELDS_THREADS
#define MHS_FIELDS_THREADS 256
#endif
constexpr int kFY = MHS_FIELDS_TILE_Y;
constexpr int kFThreads = MHS_FIELDS_THREADS;
// bottom solver: one workgroup per item.
constexpr int kBottomThreads = 1024;
// largest coarsest-grid system solved by the dense inverse
constexpr int kMaxCoarse = 1024;

// Convergence state of one solve, updated only by the finalize kernel.
struct SolveState {
    double r0;        // ||r_0||_2
    double rnorm;     // ||r_c||_2 of the last checked iterate
    double rtol;      // stopping tolerance (relative)
    int32_t checks;   // number of norms checked so far (iterate index + 1)
    int32_t done;     // 0 running, 1 converged, 2 iteration cap, 3 diverged
    int32_t max_iter; // iteration cap
    int32_t pad;
};

enum DoneCode : int32_t { kRunning = 0, kConverged = 1, kMaxed = 2, kDiverged = 3 };

// One (request, level) item of a stencil launch.
struct LevelItem {
    const void *u_in;   // iterate read by the stage
    void *u_out;        // iterate written (smoother, refinement) / coarse rhs (restriction)
    const void *f;      // right-hand side, nullptr = 0
    const void *ec;     // coarse correction added before smoothing, or FP32 e (refinement)
    void *r_out;        // refinement: FP32 residual output
    const void *coef;   // per-plane {cx, cy, d, 1/d} in the stage's arithmetic type
    double cz;          // z coupling 1/dz^2 (0 for the 2D problem)
    SolveState *state;  // stage is skipped once state->done != 0 (may be null)
    double *partials;   // per-tile sums of squared residuals (may be null)
    int32_t nx, ny, nz; // nodes of this level (nz = 1 for the 2D problem)
    int32_t ncx, ncy, ncz; // nodes of the next coarser level
    int32_t ntx, nty, ntz; // tiles per axis
    int32_t tile_base;     // first global tile of this item in its launch
    int32_t kz;            // planes per workgroup (smoother: fine planes, restriction: coarse planes)
    int32_t spread;        // read on a launch's first item: 1 = its tiles go to the XCDs in turn
                           // (items of several shapes), 0 = in contiguous ranges per XCD
};

// One request of the bottom solver: a full V-cycle from level `top` of the
// bottom hierarchy to the coarsest grid, in FP64, by a single workgroup whose
// work arrays all live in LDS (offsets in doubles into dynamic shared memory).
struct BottomItem {
    const void *f_top;            // right-hand side at the top bottom level (storage type)
    void *u_top;                  // correction written back (storage type)
    const double *coef[kMaxLevels];
    double cz[kMaxLevels];
    int32_t n[kMaxLevels][3];
    int32_t off_u[kMaxLevels];    // LDS offsets (doubles)
    int32_t off_f[kMaxLevels];
    int32_t off_c[kMaxLevels];    // LDS copy of the level's coefficient table (4 * nz)
    int32_t off_r;
    int32_t nlev;
    int32_t m;                    // unknowns of the coarsest grid
    int32_t nu1, nu2;
    int32_t planar;               // 1 = 2D problem
    const double *minv;           // m x m inverse of the coarsest operator
    SolveState *state;
};

// Largest LDS footprint of a bottom hierarchy (u, f and coefficients per
// level, r for the top level).
constexpr int kBottomLdsMax = 160 * 1024;

struct FinalizeItem {
    const double *partials;
    int32_t n;
    int32_t pad;
    SolveState *state;
};

struct FieldsItem {
    const double *P;
    double *Bx, *By, *Bz, *p, *rho;
    const double *tab; // 4 * nz: xi, dxi, pb, rhob
    double alpha, mu0, g;
    double dx, dy, dz;
    int32_t nx, ny, nz;
    int32_t ntx, nty, ntz;
    int32_t tile_base;
    int32_t kz;
    // launched ahead of the host's status read: the recovery runs only once
    // this solve has converged with P holding its iterate (null: always)
    const SolveState *gate;
    int32_t gate_odd; // -1: P always holds it; 0/1: only after an even/odd count of cycles
    int32_t gate_min; // and only after at least this many cycles
};

// Diagnostics of an equilibrium (current density, force-balance and
// divergence residuals): one thread per (x, y) column of a z-chunk.
struct DiagItem {
    const double *Bx, *By, *Bz, *p, *rho;
    double *jx, *jy, *jz, *fres, *divb;
    double mu0, g;
    double dx, dy, dz;
    int32_t nx, ny, nz;
    int32_t kz; // planes per workgroup
};

// Field-line tracing: one thread per line (seeds and points x, y, z
// interleaved; points of step n at 3 (n nlines + l)).
struct TraceItem {
    const double *Bx, *By, *Bz;
    const double *seeds; // nlines x 3
    double *points;      // (max_steps + 1) x nlines x 3
    int32_t *count;      // points per line (>= 1)
    int32_t *status;     // 0 step cap, 1 left the box, 2 |B| <= bmin
    double lx, ly, lz;
    double dx, dy, dz;
    double ds, bmin;
    int32_t nx, ny, nz;
    int32_t nlines, max_steps;
};

// Whole-array preparation items.
struct PrepItem {
    double *P;          // 3D potential (or the base plane for 2D)
    double *twin;       // ping-pong partner whose faces must match P
    const double *bz0;  // 2D: magnetogram
    double *f2;         // 2D: right-hand side -bz0
    int32_t nx, ny, nz;
    int32_t warm;
    int32_t faces;      // 1: keep P's faces (2D: edges) as Dirichlet data
    int32_t swap;       // 3D: the zero interior goes to the twin, P's interior is left as it is
    int32_t keep;       // 3D: no interior is written (the solve's first steps read it as zero);
                        // the item covers the boundary nodes only (n = prep3_faces)
    int32_t pad;
    int64_t n;          // points covered
    int64_t base;       // first global thread of this item
};

// ---- launchers (kernels.hip) ------------------------------------------------
// `dbl` selects the arithmetic/storage type: true = double, false = float.
enum SweepFlags : int {
    kHasF = 1,      // read the right-hand side
    kZeroIn = 2,    // input iterate is zero (first sweep from a zero guess)
    kNorm = 4,      // also write per-tile ||f - A u_in||^2 partials
    kProlong = 8,   // add the interpolated coarse correction to u_in first
    kTwoSweeps = 16, // two complete sweeps in one launch (2D only)
};

// Launch flags of the 3D restriction.
enum RestrictFlags : int {
    kRestrictHasF = 1,  // read the right-hand side
    kRestrictKeepZ = 2, // the step to the coarse level halves x and y only
};

hipError_t launch_sweep3(const LevelItem *items, int nitems, int ntiles, int flags, bool dbl,
                         hipStream_t s);
hipError_t launch_sweep2(const LevelItem *items, int nitems, int ntiles, int flags, bool dbl,
                         hipStream_t s);
hipError_t launch_restrict3(const LevelItem *items, int nitems, int ntiles, bool has_f, bool keepz, bool dbl,
                            hipStream_t s);
hipError_t launch_restrict2(const LevelItem *items, int nitems, int ntiles, bool dbl,
                            hipStream_t s);
// steps that keep x and y: one thread per node (ntiles = ceil(nodes / kThreads))
hipError_t launch_restrict3_z(const LevelItem *items, int nitems, int ntiles, bool has_f, bool dbl, hipStream_t s);
hipError_t launch_prolong3_z(const LevelItem *items, int nitems, int ntiles, bool dbl, hipStream_t s);
// zero_in: the iterate's interior is read as zero (a cold start's first two
// refinement steps; only its boundary nodes are loaded)
hipError_t launch_ir3(const LevelItem *items, int nitems, int ntiles, bool has_e, bool zero_in, hipStream_t s);
hipError_t launch_bottom(const BottomItem *items, int nitems, int lds_bytes, bool dbl, hipStream_t s);
hipError_t launch_finalize(const FinalizeItem *items, int nitems, hipStream_t s);
hipError_t launch_fields(const FieldsItem *items, int nitems, int ntiles, hipStream_t s);
hipError_t launch_diag(const DiagItem &item, hipStream_t s);
hipError_t launch_trace(const TraceItem &item, hipStream_t s);
// 3D preparation: nodes per thread, and the threads an item of n nodes takes
constexpr int kPrepNodes = 4;
inline int64_t prep3_threads(int64_t n) { return (n + kPrepNodes - 1) / kPrepNodes; }
// boundary nodes of an nx x ny x nz grid (planes 0 and nz - 1, the rings between)
inline int64_t prep3_faces(int nx, int ny, int nz)
{
    return 2 * (int64_t)nx * ny + (int64_t)(nz - 2) * (2 * (int64_t)nx + 2 * (int64_t)(ny - 2));
}
hipError_t launch_prep3(const PrepItem *items, int nitems, int64_t nthreads, hipStream_t s);
hipError_t launch_prep2(const PrepItem *items, int nitems, int64_t nthreads, hipStream_t s);
hipError_t launch_copy(const double *src, double *dst, int64_t n, const SolveState *skip,
                       hipStream_t s);
// dst[0 .. bytes) = 0; dst 16-byte aligned, bytes a multiple of 16
hipError_t launch_zero(void *dst, size_t bytes, hipStream_t s);

// tile counts
inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

} // namespace mhs
