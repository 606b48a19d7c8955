// Host-side plan: the multigrid hierarchy laid out in the caller's
// workspace, coefficient tables, launch programs and the C-ABI glue.
#pragma once

#include <chrono>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mhs.h"
#include "internal.h"

namespace mhs {

enum Path : int { kF64 = 0, kF32 = 1 };

constexpr size_t kAlign = 256;

// Carves 256-byte aligned regions out of a workspace (base == nullptr:
// only counts the bytes).
struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + kAlign - 1) & ~(kAlign - 1);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct Level {
    int n[3] = {0, 0, 0}; // nx, ny, nz (nz = 1 for the 2D problem)
    double h[3] = {0, 0, 0};
    size_t N = 0;
    void *u[2] = {nullptr, nullptr}; // per path: iterate / correction
    void *t[2] = {nullptr, nullptr}; // per path: ping-pong twin
    void *f[2] = {nullptr, nullptr}; // per path: right-hand side
    double *coef64 = nullptr;        // device, 4 * nz
    float *coef32 = nullptr;         // device, 4 * nz
    double cz = 0.0;
    int st[3] = {0, 0, 0}; // smoother tiles per axis
    int rt[3] = {0, 0, 0}; // restriction tiles per axis (onto level+1)
    int kz = 1;            // smoother planes per workgroup
    int kc = 1;            // restriction coarse planes per workgroup
    // z-chunking of levels >= 1 in batched (merged) launches: fewer, longer
    // z-marches, since the merged launch has many requests' tiles
    int kz_b = 1, stz_b = 1;
    int kc_b = 1, rtz_b = 1;
    int zs = 0;            // xi of plane k is xi[k << zs] of the finest grid
    bool keepz = false;    // the step to level+1 halves x and y only
    bool keepxy = false;   // the step to level+1 halves z only
    int ity = 0;           // refinement-step tiles in y (kTY rows; the smoother's are kSTY)
    int sweep_tiles() const { return st[0] * st[1] * st[2]; }
    int ir_tiles() const { return st[0] * ity * st[2]; }
    int restrict_tiles() const { return rt[0] * rt[1] * rt[2]; }
};

struct Hierarchy {
    bool planar = false;
    int L = 0; // levels in use (the 3D depth may be cut per model)
    int b = 0; // first level handled by the bottom solver
    int Lgeo = 0, bgeo = 0; // geometric depth and bottom level (buffers are carved for these)
    int mcap = 0;           // largest coarsest-grid size the inverse buffer holds
    Level lv[kMaxLevels];
    int lds_bytes = 0;      // bottom solver LDS footprint
    bool batched = false;   // builders record launches for merging (z-chunking kz_b, kc_b)
    double *minv = nullptr; // device m x m
    int m = 0;              // coarsest unknowns
    double *partials = nullptr;
    int npart = 0;
};

// One kernel launch of a program (the device item table is in the workspace).
struct Launch {
    enum Kind {
        kSweep3, kSweep2, kRestrict3, kRestrict2, kIr3, kBottom, kFinalize, kCopy, kFields, kPrep3, kPrep2,
        kRestrict3Z, kProlong3Z,
        // the general operator (general.hip): items are GenItem
        kGenSweep, kGenResid, kGenRestrict, kGenProlong, kGenCoarsest, kZero
    } kind;
    int flags = 0;
    bool dbl = true;
    const void *items = nullptr; // device pointer
    int nitems = 1;
    int ntiles = 0;
    int lds = 0; // bottom: dynamic LDS bytes
    // copy
    const double *src = nullptr;
    double *dst = nullptr;
    int64_t n = 0; // copy: elements; prep: threads
    const SolveState *gate = nullptr; // copy: skipped once this solve is done
    int prof = -1;                    // measurement class (MHS_PROF_*), -1 = none
    double bytes = 0.0;               // compulsory HBM bytes of the launch
    bool pre = false;                 // runs before the cycle's convergence check
};

// Host staging of item tables: items are appended in host memory and copied
// to the device region in one transfer.
struct Staging {
    char *host = nullptr; // pinned
    char *dev = nullptr;  // workspace region
    size_t cap = 0, used = 0;
    hipEvent_t inflight = nullptr;
    template <typename T>
    const T *put(const T &v)
    {
        used = (used + 63) & ~size_t(63);
        if (used + sizeof(T) > cap) return nullptr;
        std::memcpy(host + used, &v, sizeof(T));
        const T *d = reinterpret_cast<const T *>(dev + used);
        used += sizeof(T);
        return d;
    }
};

// Event-bracketed launches awaiting collection.
struct ProfRecord {
    int klass;
    int cycle; // index of the cycle/step the launch belongs to (-1: always counted)
    bool pre;  // launched before that cycle's convergence check
    double bytes;
    hipEvent_t start, end;
};

struct Profiler {
    int mask = 0; // bit k set: launches of class k are timed
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    std::vector<ProfRecord> pending;
    double ms[MHS_PROF_NCLASS] = {};
    double bytes[MHS_PROF_NCLASS] = {};
    long long launches[MHS_PROF_NCLASS] = {};
};

struct Program {
    std::vector<Launch> launches;
    bool ok = true;
};

// A cycle program captured as a HIP graph.  Kernels read their work items
// from the staging area, so an executable graph stays valid for every call
// whose launches (kernel, variant, item address, grid) are the same.
struct CachedGraph {
    std::vector<Launch> launches;
    hipGraphExec_t exec = nullptr;
    unsigned long long last_use = 0;
};

struct ModelCache {
    bool valid = false;
    double alpha = 0.0;
    std::vector<double> xi;
};

} // namespace mhs

struct mhs_plan;

namespace mhs {

// ---- shared host helpers (api.cpp) ------------------------------------------
int fail(int code, const char *fmt, ...);
#define HIPCHK(expr)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return ::mhs::fail(MHS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int validate_model(const mhs_plan *p, const mhs_model *m, bool need_fields);
int validate_opts(const mhs_opts *o);
// Host copies of a model's device tables (per-level coefficients, coarsest
// inverse) with their destinations; prepare_model fills it and sets the
// plan's depth and model cache, upload_model also copies and waits.
struct ModelUpload {
    struct Part {
        void *dst;
        size_t off, bytes;
    };
    std::vector<Part> parts;
    std::vector<char> data;
};
int prepare_model(mhs_plan *p, const mhs_model *model, ModelUpload &up);
int upload_model(mhs_plan *p, const mhs_model *model, hipStream_t s);
// Forget which model the plan's tables hold (its upload did not happen).
void invalidate_model(mhs_plan *p);
int set_device(const mhs_plan *p);
SolveState initial_state(double rtol, int max_iter);
int status_of(int32_t done);

// Program builders: append launches whose item tables are put into `st`.
void add_finalize(Program &pg, Staging &st, const double *partials, int n, SolveState *state);
void *add_cycle(Program &pg, Staging &st, const Hierarchy &h, int path, void *a0, void *b0, const void *f0,
                bool first_zero, bool first_norm, int nu1, int nu2, SolveState *state);
// zero_in: uin's interior is read as zero (see launch_ir3)
void add_ir_step(Program &pg, Staging &st, const Hierarchy &h, const double *uin, double *uout, const void *e,
                 float *r32, SolveState *state, bool zero_in = false);
FieldsItem fields_item(const mhs_plan *p, const mhs_model *model, const double *tab, const double *P, double *Bx,
                       double *By, double *Bz, double *pr, double *rho);
hipError_t exec_launch(const Launch &L, hipStream_t s);
int run_program(mhs_plan *p, const Program &pg, hipStream_t s, int cycle = -1);
// Launches [begin, end) of a program.
int run_range(mhs_plan *p, const Program &pg, size_t begin, size_t end, hipStream_t s, int cycle);
// One cycle's launches: replayed as a captured graph when `graph` is set and
// no class is being profiled, else launched one by one.
int run_cycle(mhs_plan *p, const Program &pg, hipStream_t s, int cycle, bool graph);
int begin_staging(mhs_plan *p);
int flush_staging(mhs_plan *p, hipStream_t s);
int read_state(mhs_plan *p, const SolveState *d_state, SolveState *out, hipStream_t s);
// Solve kinds whose last cycle count sizes the first speculative batch.
enum SolveKind : int { kSolve2D = 0, kSolve3D64 = 1, kSolve3DMixed = 2, kSolveGeneral = 3, kSolveKinds = 4 };
// The cycles (or refinement steps) a converged solve took, with the options
// that fix how many it needs for a given problem.
struct CycleHint {
    int cycles = 0;
    double rtol = 0.0;
    int nu1 = 0, nu2 = 0, inner = 0;
    bool matches(const mhs_opts *o) const
    {
        return cycles > 0 && rtol == o->rtol && nu1 == o->nu1 && nu2 == o->nu2 && inner == o->inner_cycles;
    }
};
int next_batch(const SolveState &ss, const mhs_opts *o, int launched, int hint);
// The first batch of a solve of `kind` on plan p, and the record of a
// finished one.
int hint_of(const mhs_plan *p, int kind, const mhs_opts *o);
void record_cycles(mhs_plan *p, int kind, const mhs_opts *o, const SolveState &ss);
// `overlap`, when given, runs once on the host after the first batch of
// launches is enqueued (host work that overlaps the device's).
int drive(mhs_plan *p, const Program &cycle, const SolveState *d_state, const mhs_opts *o, SolveState *out,
          int *syncs, hipStream_t s, int kind, const std::function<int()> *overlap = nullptr);
double seconds_since(std::chrono::steady_clock::time_point t0);

// Shapes and step kinds of a multigrid hierarchy (api.cpp).
int build_geometry(Hierarchy &h, const int n0[3], const double len[3], bool planar);

// ---- the general operator (general.hip) -----------------------------------
struct GenPlan;
// Geometry of the general problems' hierarchies (3D and the three face
// orientations) and their buffers; base == nullptr only counts bytes.
void gen_create(mhs_plan *p, Carver &cv);
struct GenPlanDeleter {
    void operator()(GenPlan *g) const;
};
hipError_t gen_exec(const Launch &L, hipStream_t s);
// Next timing event of the profiler's pool (created on first use); nullptr on failure.
hipEvent_t prof_event(Profiler &pr);

} // namespace mhs

struct mhs_plan {
    mhs_grid grid{};
    int precisions = 0;
    int device = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    mhs::Hierarchy h3, h2;
    // the FP64 twin of the level-0 potential (3D) and the 2D base plane
    mhs::SolveState *d_states = nullptr; // [0] 2D, [1] 3D, [2] stage
    mhs::SolveState *h_states = nullptr; // pinned mirror
    double *d_fields_tab = nullptr;      // 4 * nz
    mhs::Staging stage;
    mhs::ModelCache cache;
    double *d_scratch_norm = nullptr;    // stage residual-norm partials
    int scratch_npart = 0;
    mhs::Profiler prof;
    std::unique_ptr<mhs::GenPlan, mhs::GenPlanDeleter> gen; // the general operator (MHS_PLAN_GENERAL)
    // cycle programs captured as graphs (capture stream created on first use)
    bool graphs_ok = true;
    hipStream_t cap = nullptr;
    std::vector<mhs::CachedGraph> graphs;
    unsigned long long graph_clock = 0;
    // cycles (or refinement steps) the last converged solve of each kind
    // took: the next solve with the same options launches that many plus
    // the checking one in its first batch
    mhs::CycleHint last_cycles[mhs::kSolveKinds];
};
