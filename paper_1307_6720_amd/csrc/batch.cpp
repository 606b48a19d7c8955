// Continuous batching of independent equilibria.
//
// Every request runs the procedure of Section 2.2 (the lower-boundary solve
// of (11), the interior solve of (8), the field recovery) on its own plan.
// A tick advances each active request by one V-cycle (or one refinement
// step) of its current phase.  The per-request programs are built with the
// same builders as the single-request entry points into a host recorder,
// tagged with a merge key, and launches with equal key and kernel variant
// are fused into one multi-item launch whose descriptor table lists the
// requests' items back to back (tile offsets prefix-summed).  Kernels find
// their item by binary search over those offsets, so each request keeps its
// own tiling and reduction order: results are bitwise those of the
// single-request path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "plan.h"

using namespace mhs;

namespace {

constexpr int kMaxBatchSlots = 1024;
constexpr size_t kWsAlign = 256;
// Descriptor bytes one request may use per tick (default options need
// about 6 KB at 257^3; nu1 = nu2 = 16 with several inner cycles do not fit).
constexpr size_t kSlotStageBytes = 48 * 1024;
constexpr size_t kItemAlign = 64;

enum Phase : int { kFree = 0, kBoundary, kInterior, kFinish, kDone };

struct Slot {
    Phase phase = kFree;
    bool fresh = false;       // the current phase starts in the next tick
    bool finish_sent = false; // the field recovery is launched (kFinish)
    int64_t epoch = 0;        // identifies the current phase of the current request
    mhs_plan *plan = nullptr;
    double alpha = 0.0, mu0 = 1.0, g = 1.0;
    const double *bz0 = nullptr;
    double *P = nullptr, *Bx = nullptr, *By = nullptr, *Bz = nullptr, *p = nullptr, *rho = nullptr;
    mhs_opts opts{};
    int steps = 0; // programs launched in the current phase
    // mixed interior phase: the iterate starts in P's twin (the plan's last
    // converged count was odd, so the same count ends in P without a copy)
    bool swap = false;
    int ticks = 0; // ticks of the current phase whose status was read
    mhs_info info[2]{};
    std::chrono::steady_clock::time_point t0;
    // the model's device tables, copied on the tick that first launches the
    // request (admission does not touch the device)
    ModelUpload up;
    bool upload_pending = false;
    size_t bytes = 0; // device footprint counted against the batch's budget
};

// One launch of one request's program with its merge key.
struct Rec {
    int64_t key;
    int slot;
    Launch L;
};

// Keys order the launches of a tick.  A request's program is a prologue
// followed by one or more V-cycles (segments).  Within a cycle, launches
// before the bottom solve are numbered from the top and launches after it
// from the end, so equal stages of requests whose hierarchies differ in
// depth share a key.  Keys increase along every request's program, so
// sorting by key keeps each request's own order.
constexpr int kPartShift = 16;
constexpr int kMaxPos = (1 << kPartShift) - 1;
enum Part : int { kPrologue = 0, kDescent = 1, kBottomPart = 2, kAscent = 3, kEpilogue = 4 };

int64_t key_of(int seg, int part, int pos) { return ((int64_t)seg * 8 + part) << kPartShift | pos; }

void tag_cycle(const Program &pg, int seg, int slot, std::vector<Rec> &out)
{
    const size_t n = pg.launches.size();
    size_t ib = n;
    for (size_t i = 0; i < n; ++i)
        if (pg.launches[i].kind == Launch::kBottom) {
            ib = i;
            break;
        }
    int asc = 0;
    for (size_t i = ib + 1; i < n; ++i)
        if (pg.launches[i].kind != Launch::kCopy) ++asc;
    int j = 0, c = 0;
    for (size_t i = 0; i < n; ++i) {
        const Launch &L = pg.launches[i];
        int64_t k;
        if (i < ib)
            k = key_of(seg, kDescent, (int)i);
        else if (i == ib)
            k = key_of(seg, kBottomPart, 0);
        else if (L.kind == Launch::kCopy)
            k = key_of(seg, kEpilogue, c++);
        else
            k = key_of(seg, kAscent, kMaxPos - (asc - 1 - j++));
        out.push_back({k, slot, L});
    }
}

void tag_one(const Launch &L, int64_t key, int slot, std::vector<Rec> &out) { out.push_back({key, slot, L}); }

// Profiling of merged launches: one event pair per launch, and per item the
// slot, whether it runs before its cycle's convergence check, and its
// compulsory bytes.  After the tick's status read-back an item counts if it
// ran: it precedes the check, or its request did not stop at this tick.
struct ProfItem {
    int slot;
    bool pre;
    double bytes;
};
struct BatchProf {
    int klass;
    size_t first, count; // items
    hipEvent_t start, end;
};

// What a tick launched for one slot: the phase and its epoch.  When the
// tick's status is read, it applies to the slot only if the slot is still
// in that phase (the epoch matches).
struct Snap {
    bool launched = false;
    Phase phase = kFree;
    int64_t epoch = 0;
};

// Buffers of one tick in flight.  Ticks alternate between two of them:
// tick t is built and launched while tick t-1 still runs, and tick t-1's
// status is read after that, so the host's work for a tick overlaps the
// device's work for the previous one.
struct Tick {
    Staging stage;                  // merged descriptor tables (pinned host + workspace)
    char *upload = nullptr;         // pinned: model tables of requests starting in this tick
    size_t upload_cap = 0;
    SolveState *h_init = nullptr;   // pinned: fresh status words to upload
    SolveState *h_read = nullptr;   // pinned: status words read back
    hipEvent_t done = nullptr;      // after the read-back
    bool live = false;              // launched, status not yet read
    int top = 0;                    // one past the highest slot launched
    std::vector<Snap> snap;
    std::vector<ProfItem> prof_items;
    std::vector<BatchProf> prof_pending;
};

} // namespace

struct mhs_batch {
    int max_slots = 0;
    int device = 0;
    size_t budget = 0;  // HBM budget of the admitted requests (0 = none)
    size_t in_use = 0;  // footprint of the slots not yet released
    SolveState *d_states = nullptr; // per slot, in the workspace
    Tick ticks[2];
    int64_t tick_no = 0;            // ticks launched
    int64_t epochs = 0;             // phase epochs handed out
    std::vector<char> rec_buf;      // host recorder of per-request items (one tick)
    Staging rec;
    std::vector<Slot> slots;
    std::vector<Rec> recs;
    Profiler prof;                  // class mask and totals (events: per tick, below)
    std::vector<hipEvent_t> ev_pool[2];
};

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t states_bytes(int max_slots) { return align_up((size_t)max_slots * sizeof(SolveState), kWsAlign); }
size_t stage_bytes(int max_slots) { return (size_t)max_slots * kSlotStageBytes; }
constexpr int kTicksInFlight = 2;

// A recorder is a Staging whose "device" side is its own host buffer: the
// builders put items there and Launch::items points at them.
void reset_recorder(mhs_batch *b)
{
    b->rec.host = b->rec_buf.data();
    b->rec.dev = b->rec_buf.data();
    b->rec.cap = b->rec_buf.size();
    b->rec.used = 0;
}

// Append the launches of slot `i` for its current phase to `out`.
// Records a plan's launches with the batched z-chunking of its 3D levels
// >= 1 for as long as it lives.
struct BatchedTiling {
    Hierarchy &h;
    explicit BatchedTiling(Hierarchy &hh) : h(hh) { h.batched = true; }
    ~BatchedTiling() { h.batched = false; }
};

bool build_slot(const Slot &S, int i, SolveState *state, Staging &R, std::vector<Rec> &out)
{
    mhs_plan *p = S.plan;
    BatchedTiling tiling(p->h3);
    const mhs_opts &o = S.opts;
    if (S.phase == kBoundary) {
        Hierarchy &h = p->h2;
        if (S.fresh) {
            PrepItem pi{};
            pi.P = S.P;
            pi.twin = (double *)h.lv[0].t[kF64];
            pi.bz0 = S.bz0;
            pi.f2 = (double *)h.lv[0].f[kF64];
            pi.nx = p->grid.nx;
            pi.ny = p->grid.ny;
            pi.nz = 1;
            pi.warm = o.warm_start;
            pi.faces = o.faces;
            pi.n = (int64_t)p->grid.nx * p->grid.ny;
            const PrepItem *d = R.put(pi);
            if (!d) return false;
            Launch L{};
            L.kind = Launch::kPrep2;
            L.items = d;
            L.n = pi.n;
            tag_one(L, key_of(0, kPrologue, 0), i, out);
        }
        Program pg;
        void *res = add_cycle(pg, R, h, kF64, S.P, h.lv[0].t[kF64], h.lv[0].f[kF64], false, true, o.nu1, o.nu2,
                              state);
        if (res != (void *)S.P) {
            Launch c{};
            c.kind = Launch::kCopy;
            c.src = (const double *)res;
            c.dst = S.P;
            c.n = (int64_t)p->grid.nx * p->grid.ny;
            c.gate = state;
            pg.launches.push_back(c);
        }
        if (!pg.ok) return false;
        tag_cycle(pg, 0, i, out);
        return true;
    }
    if (S.phase == kInterior) {
        Hierarchy &h = p->h3;
        const Level &l0 = h.lv[0];
        double *T0 = (double *)l0.t[kF64];
        const int64_t N = (int64_t)l0.N;
        if (S.fresh) {
            PrepItem pi{};
            pi.P = S.P;
            pi.twin = T0;
            pi.nx = p->grid.nx;
            pi.ny = p->grid.ny;
            pi.nz = p->grid.nz;
            pi.warm = o.warm_start;
            pi.faces = o.faces;
            pi.swap = S.swap ? 1 : 0;
            // a mixed cold start zeroes no interior (its first two steps
            // read the start iterate's interior as zero)
            pi.keep = (o.precision == MHS_PREC_MIXED && !o.warm_start) ? 1 : 0;
            pi.n = pi.keep ? prep3_faces(pi.nx, pi.ny, pi.nz) : N;
            const PrepItem *d = R.put(pi);
            if (!d) return false;
            Launch L{};
            L.kind = Launch::kPrep3;
            L.items = d;
            L.n = prep3_threads(pi.n); // threads (base of the merged launch counts threads)
            tag_one(L, key_of(0, kPrologue, 0), i, out);
        }
        if (o.precision == MHS_PREC_FP64) {
            Program pg;
            void *res = add_cycle(pg, R, h, kF64, S.P, T0, nullptr, false, true, o.nu1, o.nu2, state);
            if (res != (void *)S.P) {
                Launch c{};
                c.kind = Launch::kCopy;
                c.src = (const double *)res;
                c.dst = S.P;
                c.n = N;
                c.gate = state;
                pg.launches.push_back(c);
            }
            if (!pg.ok) return false;
            tag_cycle(pg, 0, i, out);
            return true;
        }
        // refinement step S.steps: step 0 checks U; odd steps write U + e
        // into V, even steps V + e into U (the single-request ping-pong; U
        // is P and V its twin, or the other way round with S.swap)
        float *r32 = (float *)l0.f[kF32];
        std::vector<Program> inner((size_t)o.inner_cycles);
        void *ebuf = nullptr;
        for (int c = 0; c < o.inner_cycles; ++c) {
            void *a = c == 0 ? l0.u[kF32] : ebuf;
            void *bb = (a == l0.u[kF32]) ? l0.t[kF32] : l0.u[kF32];
            ebuf = add_cycle(inner[(size_t)c], R, h, kF32, a, bb, r32, c == 0, false, o.nu1, o.nu2, state);
        }
        const int s = S.steps;
        double *U = S.swap ? T0 : S.P, *V = S.swap ? S.P : T0;
        const double *uin = (s == 0 || (s & 1)) ? U : V;
        double *uout = s == 0 ? nullptr : ((s & 1) ? V : U);
        Program ir;
        add_ir_step(ir, R, h, uin, uout, s == 0 ? nullptr : ebuf, r32, state, s <= 1 && !o.warm_start);
        if (!ir.ok || ir.launches.size() != 2) return false;
        tag_one(ir.launches[0], key_of(0, kPrologue, 1), i, out);
        tag_one(ir.launches[1], key_of(0, kPrologue, 2), i, out);
        for (int c = 0; c < o.inner_cycles; ++c) {
            if (!inner[(size_t)c].ok) return false;
            tag_cycle(inner[(size_t)c], c, i, out);
        }
        return true;
    }
    if (S.phase == kFinish) {
        const int64_t N = (int64_t)p->h3.lv[0].N;
        // the iterate ends in V after an odd step count, else in U; a cold
        // start that stopped at step 0 never wrote an interior: P's is zeroed
        if (o.precision == MHS_PREC_MIXED && !o.warm_start && S.info[1].cycles == 0) {
            PrepItem pi{};
            pi.P = S.P;
            pi.twin = (double *)p->h3.lv[0].t[kF64];
            pi.nx = p->grid.nx;
            pi.ny = p->grid.ny;
            pi.nz = p->grid.nz;
            pi.faces = o.faces;
            pi.n = N;
            const PrepItem *d = R.put(pi);
            if (!d) return false;
            Launch L{};
            L.kind = Launch::kPrep3;
            L.items = d;
            L.n = prep3_threads(N);
            tag_one(L, key_of(0, kPrologue, 0), i, out);
        } else if (o.precision == MHS_PREC_MIXED && ((S.info[1].cycles & 1) != (S.swap ? 1 : 0))) {
            Launch c{};
            c.kind = Launch::kCopy;
            c.src = (const double *)p->h3.lv[0].t[kF64];
            c.dst = S.P;
            c.n = N;
            tag_one(c, key_of(0, kPrologue, 0), i, out);
        }
        mhs_model m{};
        m.alpha = S.alpha;
        m.mu0 = S.mu0;
        m.g = S.g;
        const FieldsItem fi = fields_item(p, &m, p->d_fields_tab, S.P, S.Bx, S.By, S.Bz, S.p, S.rho);
        const FieldsItem *d = R.put(fi);
        if (!d) return false;
        Launch L{};
        L.kind = Launch::kFields;
        L.items = d;
        L.ntiles = fi.ntx * fi.nty * fi.ntz;
        tag_one(L, key_of(0, kDescent, 0), i, out);
        return true;
    }
    return true;
}

size_t item_size(Launch::Kind k)
{
    switch (k) {
    case Launch::kSweep3:
    case Launch::kSweep2:
    case Launch::kRestrict3:
    case Launch::kRestrict2:
    case Launch::kIr3:
    case Launch::kRestrict3Z:
    case Launch::kProlong3Z:
        return sizeof(LevelItem);
    case Launch::kBottom:
        return sizeof(BottomItem);
    case Launch::kFinalize:
        return sizeof(FinalizeItem);
    case Launch::kFields:
        return sizeof(FieldsItem);
    case Launch::kPrep3:
    case Launch::kPrep2:
        return sizeof(PrepItem);
    case Launch::kCopy:
        return 0;
    default: // the general operator's launches are never batched
        return 0;
    }
}

// Compulsory bytes of a finest-level launch from which a request's
// finest-level launches are kept out of launches merged with requests of
// another shape (at 257^3 a sweep moves 136-212 MB, at 129^3 17-27 MB).
#ifndef MHS_RUN_BYTES
#define MHS_RUN_BYTES 64e6
#endif
constexpr double kRunBytes = MHS_RUN_BYTES;

bool same_variant(const Launch &a, const Launch &b)
{
    return a.kind == b.kind && a.flags == b.flags && a.dbl == b.dbl;
}

// Fuse recs[lo, hi) (one key, one variant, distinct slots) into one launch
// whose descriptor table is written into the batch staging area.
bool merge(Staging &st, const std::vector<const Rec *> &grp, Launch *out)
{
    const Launch &first = grp[0]->L;
    const size_t sz = item_size(first.kind);
    st.used = align_up(st.used, kItemAlign);
    if (st.used + sz * grp.size() > st.cap) return false;
    char *host = st.host + st.used;
    Launch M = first;
    M.items = st.dev + st.used;
    M.nitems = (int)grp.size();
    M.ntiles = 0;
    M.lds = 0;
    M.n = 0;
    for (size_t q = 0; q < grp.size(); ++q) {
        const Launch &L = grp[q]->L;
        char *dst = host + q * sz;
        std::memcpy(dst, L.items, sz);
        switch (L.kind) {
        case Launch::kSweep3:
        case Launch::kSweep2:
        case Launch::kRestrict3:
        case Launch::kRestrict2:
        case Launch::kIr3:
        case Launch::kRestrict3Z:
        case Launch::kProlong3Z:
            reinterpret_cast<LevelItem *>(dst)->tile_base = M.ntiles;
            M.ntiles += L.ntiles;
            break;
        case Launch::kFields:
            reinterpret_cast<FieldsItem *>(dst)->tile_base = M.ntiles;
            M.ntiles += L.ntiles;
            break;
        case Launch::kPrep3:
        case Launch::kPrep2:
            reinterpret_cast<PrepItem *>(dst)->base = M.n;
            M.n += L.n;
            break;
        case Launch::kBottom:
            M.lds = std::max(M.lds, L.lds);
            break;
        default:
            break;
        }
    }
    switch (first.kind) {
    case Launch::kSweep3:
    case Launch::kSweep2:
    case Launch::kRestrict3:
    case Launch::kRestrict2:
    case Launch::kIr3:
    case Launch::kRestrict3Z:
    case Launch::kProlong3Z: {
        LevelItem *i0 = reinterpret_cast<LevelItem *>(host);
        for (size_t q = 1; q < grp.size(); ++q) {
            const LevelItem *iq = reinterpret_cast<const LevelItem *>(host + q * sz);
            if (iq->nx != i0->nx || iq->ny != i0->ny || iq->nz != i0->nz) i0->spread = 1;
        }
        break;
    }
    default:
        break;
    }
    st.used += sz * grp.size();
    *out = M;
    return true;
}

bool active(Phase ph) { return ph == kBoundary || ph == kInterior || ph == kFinish; }

int check_slot(const mhs_batch *b, int32_t slot)
{
    if (!b) return fail(MHS_ERR_INVALID_ARG, "batch is NULL");
    if (slot < 0 || slot >= b->max_slots) return fail(MHS_ERR_INVALID_ARG, "slot %d out of range", slot);
    return MHS_OK;
}

} // namespace

extern "C" {

int mhs_batch_workspace_bytes(int32_t max_slots, size_t *bytes)
{
    if (!bytes) return fail(MHS_ERR_INVALID_ARG, "bytes is NULL");
    if (max_slots < 1 || max_slots > kMaxBatchSlots)
        return fail(MHS_ERR_INVALID_ARG, "max_slots must be in 1..%d", kMaxBatchSlots);
    *bytes = states_bytes(max_slots) + kTicksInFlight * stage_bytes(max_slots);
    return MHS_OK;
}

int mhs_batch_create(int32_t max_slots, size_t hbm_budget, void *d_ws, size_t ws_bytes, mhs_batch **out)
{
    if (!out) return fail(MHS_ERR_INVALID_ARG, "batch output is NULL");
    *out = nullptr;
    size_t need = 0;
    int st = mhs_batch_workspace_bytes(max_slots, &need);
    if (st) return st;
    if (!d_ws || ((uintptr_t)d_ws % kWsAlign) != 0)
        return fail(MHS_ERR_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < need) return fail(MHS_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    mhs_batch *b = new mhs_batch();
    b->max_slots = max_slots;
    b->budget = hbm_budget;
    b->slots.resize((size_t)max_slots);
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return fail(MHS_ERR_HIP, "hipGetDevice failed");
    }
    b->d_states = (SolveState *)d_ws;
    b->rec_buf.resize(stage_bytes(max_slots));
    for (int k = 0; k < kTicksInFlight; ++k) {
        Tick &t = b->ticks[k];
        t.stage.dev = (char *)d_ws + states_bytes(max_slots) + (size_t)k * stage_bytes(max_slots);
        t.stage.cap = stage_bytes(max_slots);
        t.snap.resize((size_t)max_slots);
        if (hipHostMalloc((void **)&t.stage.host, t.stage.cap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&t.h_init, (size_t)max_slots * sizeof(SolveState), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&t.h_read, (size_t)max_slots * sizeof(SolveState), hipHostMallocDefault) !=
                hipSuccess ||
            hipEventCreateWithFlags(&t.done, hipEventDisableTiming) != hipSuccess) {
            mhs_batch_destroy(b);
            return fail(MHS_ERR_HIP, "pinned host allocation or event creation failed");
        }
    }
    *out = b;
    return MHS_OK;
}

int mhs_batch_destroy(mhs_batch *b)
{
    if (!b) return MHS_OK;
    for (Tick &t : b->ticks) {
        // a tick still in flight copies into the pinned buffers freed below
        if (t.live && t.done) (void)hipEventSynchronize(t.done);
        if (t.done) (void)hipEventDestroy(t.done);
        if (t.stage.host) (void)hipHostFree(t.stage.host);
        if (t.h_init) (void)hipHostFree(t.h_init);
        if (t.h_read) (void)hipHostFree(t.h_read);
        if (t.upload) (void)hipHostFree(t.upload);
    }
    for (auto &pool : b->ev_pool)
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    delete b;
    return MHS_OK;
}

int mhs_batch_admit(mhs_batch *b, mhs_plan *plan, const mhs_model *model, const double *d_bz0, double *d_P,
                    double *d_Bx, double *d_By, double *d_Bz, double *d_p, double *d_rho, const mhs_opts *o,
                    int32_t *slot)
{
    if (!b || !plan || !d_bz0 || !d_P || !d_Bx || !d_By || !d_Bz || !d_p || !d_rho || !slot)
        return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    int st = validate_opts(o);
    if (st) return st;
    if ((st = validate_model(plan, model, true))) return st;
    if (!(plan->precisions & o->precision))
        return fail(MHS_ERR_UNSUPPORTED, "plan was not created for precision %d", o->precision);
    if (plan->device != b->device) return fail(MHS_ERR_INVALID_ARG, "plan and batch are on different devices");
    int free_slot = -1;
    for (int i = 0; i < b->max_slots; ++i) {
        const Slot &S = b->slots[(size_t)i];
        if (S.phase != kFree && S.plan == plan)
            return fail(MHS_ERR_INVALID_ARG, "plan is already held by slot %d", i);
        if (S.phase == kFree && free_slot < 0) free_slot = i;
    }
    if (free_slot < 0) return fail(MHS_ERR_BUDGET, "no free slot (max_slots %d)", b->max_slots);
    size_t need = 0;
    if ((st = mhs_request_bytes(&plan->grid, plan->precisions, &need))) return st;
    if (b->budget && b->in_use + need > b->budget)
        return fail(MHS_ERR_BUDGET, "admission would hold %zu bytes of device memory, over the budget of %zu",
                    b->in_use + need, b->budget);
    if ((st = set_device(plan))) return st;

    Slot S{};
    S.plan = plan;
    S.alpha = model->alpha;
    S.mu0 = model->mu0;
    S.g = model->g;
    S.bz0 = d_bz0;
    S.P = d_P;
    S.Bx = d_Bx;
    S.By = d_By;
    S.Bz = d_Bz;
    S.p = d_p;
    S.rho = d_rho;
    S.opts = *o;
    // coefficient tables, coarsest inverse (this also fixes the depth of the
    // hierarchy for this model) and the field tables, prepared on the host
    if ((st = prepare_model(plan, model, S.up))) return st;
    {
        const int nz = plan->grid.nz;
        std::vector<double> tab(4 * (size_t)nz);
        std::copy(model->xi, model->xi + nz, tab.begin());
        std::copy(model->dxi, model->dxi + nz, tab.begin() + nz);
        std::copy(model->pb, model->pb + nz, tab.begin() + 2 * nz);
        std::copy(model->rhob, model->rhob + nz, tab.begin() + 3 * nz);
        const size_t off = (S.up.data.size() + 63) & ~size_t(63);
        S.up.data.resize(off + tab.size() * sizeof(double));
        std::memcpy(S.up.data.data() + off, tab.data(), tab.size() * sizeof(double));
        S.up.parts.push_back({plan->d_fields_tab, off, tab.size() * sizeof(double)});
    }
    // every phase's per-tick descriptors must fit the slot's share (with
    // room for the alignment of each merged table)
    for (Phase ph : {kBoundary, kInterior, kFinish}) {
        for (int steps : {0, 1}) {
            S.phase = ph;
            S.fresh = true;
            S.steps = steps;
            reset_recorder(b);
            std::vector<Rec> tmp;
            const bool ok = build_slot(S, free_slot, b->d_states + free_slot, b->rec, tmp);
            if (!ok || b->rec.used + kItemAlign * tmp.size() > kSlotStageBytes) {
                invalidate_model(plan); // the prepared tables never reach the device
                return fail(MHS_ERR_BUDGET, "the request's per-tick launch descriptors exceed %zu bytes",
                            kSlotStageBytes);
            }
        }
    }
    S.upload_pending = true;

    S.phase = kBoundary;
    S.fresh = true;
    S.finish_sent = false;
    S.epoch = ++b->epochs;
    S.steps = 0;
    S.ticks = 0;
    S.t0 = std::chrono::steady_clock::now();
    S.bytes = need;
    b->in_use += need;
    b->slots[(size_t)free_slot] = S;
    *slot = free_slot;
    return MHS_OK;
}

int mhs_batch_step(mhs_batch *b, void *stream, int32_t *n_active)
{
    if (!b) return fail(MHS_ERR_INVALID_ARG, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != b->device) HIPCHK(hipSetDevice(b->device));
    if (n_active) *n_active = 0;

    // Tick t uses buffer t % 2, last used by tick t-2, whose status the
    // previous call read (after waiting for it).
    Tick &T = b->ticks[b->tick_no & 1];
    Tick &prev = b->ticks[(b->tick_no + 1) & 1];

    // 1. record the programs of every slot with work to launch, from the
    // phases known now (a request that stopped in the tick still in flight
    // gets one more cycle, whose launches exit at once on its status word)
    reset_recorder(b);
    b->recs.clear();
    int top = 0;
    for (int i = 0; i < b->max_slots; ++i) {
        Slot &S = b->slots[(size_t)i];
        Snap &sn = T.snap[(size_t)i];
        sn.launched = false;
        if (!active(S.phase) || (S.phase == kFinish && S.finish_sent)) continue;
        top = i + 1;
        if (S.fresh && S.phase != kFinish) T.h_init[i] = initial_state(S.opts.rtol, S.opts.max_cycles);
        if (!build_slot(S, i, b->d_states + i, b->rec, b->recs))
            return fail(MHS_ERR_WORKSPACE, "descriptor recorder exhausted");
        sn.launched = true;
        sn.phase = S.phase;
        sn.epoch = S.epoch;
    }
    T.top = top;

    // 2. merge equal (key, variant) launches across requests
    std::stable_sort(b->recs.begin(), b->recs.end(), [](const Rec &x, const Rec &y) { return x.key < y.key; });
    std::vector<Launch> plan_launches;
    std::vector<std::pair<size_t, size_t>> launch_items; // per launch: its items in prof_items
    const bool profiling = b->prof.mask != 0;
    T.prof_items.clear();
    T.prof_pending.clear();
    auto note_items = [&](const std::vector<const Rec *> &g) {
        const size_t first = T.prof_items.size();
        if (profiling)
            for (const Rec *r : g) T.prof_items.push_back({r->slot, r->L.pre, r->L.bytes});
        launch_items.emplace_back(first, g.size());
    };
    T.stage.used = 0;
    std::vector<const Rec *> grp;
    // Finest-level launches of large requests are not merged with those of
    // requests of another shape: the tiles of a merged launch are split
    // among the XCDs in contiguous ranges, and tiles of different shapes
    // march different numbers of planes, so such a launch would leave some
    // XCDs idle while others finish the large request's tiles.  Instead a
    // request's consecutive finest-level launches (the refinement step and
    // the pre-smoothing of its first cycle; the post-smoothing of a cycle
    // and the pre-smoothing of the next) run back to back as a run of its
    // own, launched just before its request's first launch that is not part
    // of it.  Launches of requests of one shape are merged as they are.
    auto deferrable = [](const Launch &L) {
        return (L.prof == MHS_PROF_SMOOTH_L0 || L.prof == MHS_PROF_RESTRICT_L0 || L.prof == MHS_PROF_REFINE) &&
               L.bytes >= kRunBytes;
    };
    auto same_shape = [](const Launch &a, const Launch &c) {
        const LevelItem *x = reinterpret_cast<const LevelItem *>(a.items);
        const LevelItem *y = reinterpret_cast<const LevelItem *>(c.items);
        return x->nx == y->nx && x->ny == y->ny && x->nz == y->nz;
    };
    std::vector<std::vector<const Rec *>> run((size_t)b->max_slots);
    auto flush = [&](int slot) {
        for (const Rec *r : run[(size_t)slot]) {
            grp.assign(1, r);
            Launch M{};
            if (!merge(T.stage, grp, &M)) return false;
            plan_launches.push_back(M);
            note_items(grp);
        }
        run[(size_t)slot].clear();
        return true;
    };
    for (size_t lo = 0; lo < b->recs.size();) {
        size_t hi = lo;
        while (hi < b->recs.size() && b->recs[hi].key == b->recs[lo].key) ++hi;
        std::vector<bool> taken(hi - lo, false);
        for (size_t a = lo; a < hi; ++a) {
            const Rec &r = b->recs[a];
            bool defer = r.L.kind == Launch::kFinalize && !run[(size_t)r.slot].empty();
            if (deferrable(r.L))
                for (size_t c = lo; c < hi && !defer; ++c)
                    defer = same_variant(b->recs[c].L, r.L) && !same_shape(b->recs[c].L, r.L);
            if (defer) {
                run[(size_t)r.slot].push_back(&r);
                taken[a - lo] = true;
            }
        }
        for (size_t a = lo; a < hi; ++a)
            if (!taken[a - lo] && !run[(size_t)b->recs[a].slot].empty() && !flush(b->recs[a].slot))
                return fail(MHS_ERR_WORKSPACE, "batch descriptor table exhausted");
        for (size_t a = lo; a < hi; ++a) {
            if (taken[a - lo]) continue;
            const Launch &La = b->recs[a].L;
            if (La.kind == Launch::kCopy) {
                plan_launches.push_back(La);
                taken[a - lo] = true;
                note_items({&b->recs[a]});
                continue;
            }
            grp.clear();
            for (size_t c = a; c < hi; ++c)
                if (!taken[c - lo] && same_variant(b->recs[c].L, La)) {
                    grp.push_back(&b->recs[c]);
                    taken[c - lo] = true;
                }
            Launch M{};
            if (!merge(T.stage, grp, &M)) return fail(MHS_ERR_WORKSPACE, "batch descriptor table exhausted");
            plan_launches.push_back(M);
            note_items(grp);
        }
        lo = hi;
    }
    for (int i = 0; i < b->max_slots; ++i)
        if (!run[(size_t)i].empty() && !flush(i)) return fail(MHS_ERR_WORKSPACE, "batch descriptor table exhausted");

    // 3. model tables of starting requests, descriptors and fresh status
    // words to the device, the launches, then the status read-back
    if (top > 0) {
        size_t up_bytes = 0;
        for (int i = 0; i < top; ++i) {
            const Slot &S = b->slots[(size_t)i];
            if (T.snap[(size_t)i].launched && S.upload_pending) up_bytes = ((up_bytes + 63) & ~size_t(63)) + S.up.data.size();
        }
        if (up_bytes > T.upload_cap) {
            // this tick buffer's last use (tick t-2) has completed
            if (T.upload) HIPCHK(hipHostFree(T.upload));
            T.upload = nullptr;
            T.upload_cap = 0;
            HIPCHK(hipHostMalloc((void **)&T.upload, up_bytes, hipHostMallocDefault));
            T.upload_cap = up_bytes;
        }
        size_t up_off = 0;
        for (int i = 0; i < top; ++i) {
            Slot &S = b->slots[(size_t)i];
            if (!T.snap[(size_t)i].launched || !S.upload_pending) continue;
            up_off = (up_off + 63) & ~size_t(63);
            std::memcpy(T.upload + up_off, S.up.data.data(), S.up.data.size());
            for (const ModelUpload::Part &q : S.up.parts)
                HIPCHK(hipMemcpyAsync(q.dst, T.upload + up_off + q.off, q.bytes, hipMemcpyHostToDevice, s));
            up_off += S.up.data.size();
            S.upload_pending = false;
            S.up = ModelUpload{};
        }
        if (T.stage.used)
            HIPCHK(hipMemcpyAsync(T.stage.dev, T.stage.host, T.stage.used, hipMemcpyHostToDevice, s));
        for (int i = 0; i < top; ++i) {
            const Slot &S = b->slots[(size_t)i];
            if (T.snap[(size_t)i].launched && S.fresh && S.phase != kFinish)
                HIPCHK(hipMemcpyAsync(b->d_states + i, T.h_init + i, sizeof(SolveState), hipMemcpyHostToDevice, s));
        }
        std::vector<hipEvent_t> &pool = b->ev_pool[b->tick_no & 1];
        size_t ev_next = 0;
        auto event = [&]() -> hipEvent_t {
            if (ev_next == pool.size()) {
                hipEvent_t e = nullptr;
                if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
                pool.push_back(e);
            }
            return pool[ev_next++];
        };
        for (size_t q = 0; q < plan_launches.size(); ++q) {
            const Launch &L = plan_launches[q];
            const bool timed = profiling && L.prof >= 0 && ((b->prof.mask >> L.prof) & 1) != 0;
            BatchProf rec{};
            if (timed) {
                rec.klass = L.prof;
                rec.first = launch_items[q].first;
                rec.count = launch_items[q].second;
                rec.start = event();
                rec.end = event();
                if (!rec.start || !rec.end) return fail(MHS_ERR_HIP, "event creation failed");
                HIPCHK(hipEventRecord(rec.start, s));
            }
            const hipError_t e = exec_launch(L, s);
            if (e != hipSuccess) return fail(MHS_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
            if (timed) {
                HIPCHK(hipEventRecord(rec.end, s));
                T.prof_pending.push_back(rec);
            }
        }
        HIPCHK(hipMemcpyAsync(T.h_read, b->d_states, (size_t)top * sizeof(SolveState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(T.done, s));
        T.live = true;
        for (int i = 0; i < top; ++i) {
            Slot &S = b->slots[(size_t)i];
            if (!T.snap[(size_t)i].launched) continue;
            S.fresh = false;
            S.steps += 1;
            if (S.phase == kFinish) S.finish_sent = true;
        }
    }
    b->tick_no += 1;

    // 4. read the previous tick's status (the device is now busy with this
    // tick) and advance the phases of the requests it covered
    if (prev.live) {
        HIPCHK(hipEventSynchronize(prev.done));
        prev.live = false;
        // a slot's status applies while the slot is still in the phase the
        // tick launched (the epoch matches)
        auto current = [&](int i) {
            const Snap &sn = prev.snap[(size_t)i];
            return sn.launched && b->slots[(size_t)i].epoch == sn.epoch;
        };
        if (!prev.prof_pending.empty()) {
            std::vector<char> ran_all((size_t)prev.top, 0), ran_pre((size_t)prev.top, 0);
            for (int i = 0; i < prev.top; ++i) {
                if (!current(i)) continue; // its launches exited at once
                const Snap &sn = prev.snap[(size_t)i];
                const bool stopped = (sn.phase == kBoundary || sn.phase == kInterior) && prev.h_read[i].done != kRunning;
                ran_pre[(size_t)i] = 1;
                ran_all[(size_t)i] = stopped ? 0 : 1;
            }
            for (const BatchProf &r : prev.prof_pending) {
                double bytes = 0.0;
                bool ran = false;
                for (size_t k = r.first; k < r.first + r.count; ++k) {
                    const ProfItem &it = prev.prof_items[k];
                    if (it.pre ? ran_pre[(size_t)it.slot] : ran_all[(size_t)it.slot]) {
                        bytes += it.bytes;
                        ran = true;
                    }
                }
                if (!ran) continue;
                float ms = 0.0f;
                HIPCHK(hipEventElapsedTime(&ms, r.start, r.end));
                b->prof.ms[r.klass] += ms;
                b->prof.bytes[r.klass] += bytes;
                b->prof.launches[r.klass] += 1;
            }
            prev.prof_pending.clear();
        }
        for (int i = 0; i < prev.top; ++i) {
            if (!current(i)) continue;
            Slot &S = b->slots[(size_t)i];
            S.ticks += 1;
            if (S.phase == kFinish) {
                S.phase = kDone;
                S.epoch = ++b->epochs;
                continue;
            }
            const SolveState &ss = prev.h_read[i];
            if (ss.done == kRunning) continue;
            const int q = S.phase == kBoundary ? 0 : 1;
            mhs_info &inf = S.info[q];
            inf.status = status_of(ss.done);
            inf.cycles = std::max(0, ss.checks - 1);
            inf.inner_cycles = (q == 1 && S.opts.precision == MHS_PREC_MIXED) ? inf.cycles * S.opts.inner_cycles : 0;
            inf.host_syncs = S.ticks;
            inf.r0 = ss.r0;
            inf.rel_residual = ss.r0 > 0 ? ss.rnorm / ss.r0 : 0.0;
            inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - S.t0).count();
            S.epoch = ++b->epochs;
            if (q == 1 && S.opts.precision == MHS_PREC_MIXED) record_cycles(S.plan, kSolve3DMixed, &S.opts, ss);
            if (inf.status != MHS_OK) {
                S.phase = kDone;
                continue;
            }
            if (q == 0)
                S.swap = S.opts.precision == MHS_PREC_MIXED && !S.opts.warm_start &&
                         (hint_of(S.plan, kSolve3DMixed, &S.opts) & 1);
            S.phase = q == 0 ? kInterior : kFinish;
            S.fresh = true;
            S.finish_sent = false;
            S.steps = 0;
            S.ticks = 0;
        }
    }
    int running = 0;
    for (const Slot &S : b->slots)
        if (active(S.phase)) ++running;
    if (n_active) *n_active = running;
    return MHS_OK;
}

int mhs_batch_poll(mhs_batch *b, int32_t slot, int32_t *done, mhs_info *boundary, mhs_info *interior)
{
    int st = check_slot(b, slot);
    if (st) return st;
    const Slot &S = b->slots[(size_t)slot];
    if (S.phase == kFree) return fail(MHS_ERR_INVALID_ARG, "slot %d is free", slot);
    if (done) *done = S.phase == kDone ? 1 : 0;
    if (boundary) *boundary = S.info[0];
    if (interior) *interior = S.info[1];
    return MHS_OK;
}

int mhs_batch_profile_enable(mhs_batch *b, int32_t class_mask)
{
    if (!b) return fail(MHS_ERR_INVALID_ARG, "batch is NULL");
    if (class_mask & ~MHS_PROF_ALL) return fail(MHS_ERR_INVALID_ARG, "unknown profiling class in mask 0x%x", class_mask);
    b->prof.mask = class_mask;
    return MHS_OK;
}

int mhs_batch_profile_read(mhs_batch *b, int32_t klass, double *total_ms, int64_t *launches, double *bytes,
                           int32_t reset)
{
    if (!b) return fail(MHS_ERR_INVALID_ARG, "batch is NULL");
    if (klass < 0 || klass >= MHS_PROF_NCLASS) return fail(MHS_ERR_INVALID_ARG, "class %d out of range", klass);
    if (total_ms) *total_ms = b->prof.ms[klass];
    if (launches) *launches = b->prof.launches[klass];
    if (bytes) *bytes = b->prof.bytes[klass];
    if (reset)
        for (int k = 0; k < MHS_PROF_NCLASS; ++k) {
            b->prof.ms[k] = 0.0;
            b->prof.bytes[k] = 0.0;
            b->prof.launches[k] = 0;
        }
    return MHS_OK;
}

int mhs_batch_release(mhs_batch *b, int32_t slot)
{
    int st = check_slot(b, slot);
    if (st) return st;
    Slot &S = b->slots[(size_t)slot];
    if (S.phase != kFree && S.upload_pending) invalidate_model(S.plan); // its tables never reached the device
    b->in_use -= S.bytes;
    b->slots[(size_t)slot] = Slot{};
    return MHS_OK;
}

int mhs_batch_bytes_in_use(const mhs_batch *b, size_t *bytes)
{
    if (!b || !bytes) return fail(MHS_ERR_INVALID_ARG, "NULL argument");
    *bytes = b->in_use;
    return MHS_OK;
}

} // extern "C"
