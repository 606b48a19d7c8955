/*
 * mhs.h -- C ABI of libmhs, a gfx950 (MI355X) multigrid solver for the
 * poloidal potential P of the NR99 linear magnetohydrostatic model, as
 * reduced to scalar elliptic problems in Section 2.2 of MacTaggart et al.,
 * "Non-symmetric magnetohydrostatic equilibria: a multigrid approach".
 *
 * Problems solved (second-order central differences, uniform grid):
 *   lower boundary, equation (11):  P_xx + P_yy = -Bz0(x, y) on z = 0,
 *                                   P = 0 on the edges of the base;
 *   interior, equation (8):  (1 - xi(z)) (P_xx + P_yy) + P_zz + alpha^2 P = 0,
 *                            P(z=0) from (11), P = 0 on top and side faces;
 * then B from equation (5) with T = alpha P (6), p from (9), rho from (10).
 *
 * Conventions shared by every entry point
 *   Grid.     nx, ny, nz nodes per axis, each 2^L + 1 with L >= 2; node
 *             spacing d = l / (n - 1); nodes run from 0 to l inclusive.
 *   Layout.   every 3D array is contiguous, x fastest:
 *             idx = i + nx * (j + ny * k)  (a torch tensor of shape
 *             (nz, ny, nx)); 2D arrays are (ny, nx), x fastest.
 *   Memory.   "d_" pointers are device pointers on the plan's device,
 *             owned by the caller.  Model arrays (xi, dxi, pb, rhob) are
 *             host pointers of length nz, copied during the call.
 *   Streams.  `stream` is a hipStream_t (NULL = the default stream).  Work is
 *             stream-ordered.  The solve entry points return once the
 *             stopping rule has been decided (they read back an 8-byte
 *             status); mhs_fields and the stage entry points are
 *             asynchronous.  A plan must not be used by two calls at once.
 *   Errors.   every function returns 0 (MHS_OK) or a positive MHS_ERR_*
 *             code; nothing throws across the ABI.  mhs_last_error()
 *             returns a thread-local message for the last failure.
 *
 * The library allocates no device memory: the caller passes a workspace
 * of mhs_workspace_bytes() bytes to mhs_plan_create(), and the plan owns
 * that memory's contents until mhs_plan_destroy().  Host-side plan
 * structures and a small pinned status buffer are allocated by
 * mhs_plan_create().
 */
#ifndef MHS_H
#define MHS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MHS_OK 0
#define MHS_ERR_INVALID_ARG 1    /* null pointer, bad option value          */
#define MHS_ERR_GRID 2           /* an axis is not 2^L+1 nodes (L >= 2), or over 2e9 nodes */
#define MHS_ERR_NOT_ELLIPTIC 3   /* xi(z_k) >= 1 at an interior plane (8)   */
#define MHS_ERR_INDEFINITE 4     /* alpha^2 too close to the spectrum of (8) */
#define MHS_ERR_NO_CONVERGENCE 5 /* max_cycles reached; P holds last iterate */
#define MHS_ERR_DIVERGED 6       /* residual non-finite or grew tenfold     */
#define MHS_ERR_BUDGET 7         /* serving: no slot or workspace too small */
#define MHS_ERR_WORKSPACE 8      /* workspace too small or misaligned       */
#define MHS_ERR_HIP 9            /* a HIP runtime call failed               */
#define MHS_ERR_UNSUPPORTED 10   /* option combination not built            */

/* ---- precisions (bit mask for plans, single value for a solve) -------- */
#define MHS_PREC_FP64 1  /* FP64 V(nu1,nu2) cycles                          */
#define MHS_PREC_MIXED 2 /* FP32 V-cycles inside FP64 iterative refinement  */
#define MHS_PLAN_GENERAL 4 /* plan mask only: the plan also serves
                              mhs_solve_general and mhs_solve_face        */

typedef struct mhs_grid {
    int32_t nx, ny, nz; /* nodes per axis, each 2^L + 1, L >= 2            */
    double lx, ly, lz;  /* box lengths (> 0)                               */
} mhs_grid;

typedef struct mhs_model {
    double alpha;      /* the constant of the field-aligned current (4)    */
    const double *xi;  /* host, nz values: xi(z_k), cross-field profile    */
    const double *dxi; /* host, nz values: dxi/dz at z_k (for (10))        */
    const double *pb;  /* host, nz values: background pressure p_b(z_k)    */
    const double *rhob;/* host, nz values: background density rho_b(z_k)   */
    double mu0;        /* permeability in the units of the model (> 0)     */
    double g;          /* gravitational acceleration (> 0)                 */
} mhs_model;

typedef struct mhs_opts {
    int32_t precision;    /* MHS_PREC_FP64 or MHS_PREC_MIXED (interior only) */
    int32_t max_cycles;   /* cap on V-cycles (FP64) or refinement steps     */
    double rtol;          /* stop when ||r||_2 / ||r_0||_2 <= rtol          */
    int32_t nu1, nu2;     /* pre/post red-black Gauss-Seidel sweeps (>= 1)  */
    int32_t inner_cycles; /* FP32 V-cycles per refinement step (mixed)      */
    int32_t warm_start;   /* 1: use P's interior as the initial guess       */
    int32_t check_every;  /* cycles launched between host status reads; 0 = adaptive */
    int32_t faces;        /* MHS_FACES_ZERO or MHS_FACES_GIVEN (below)      */
    int32_t graph;        /* 1: each cycle replayed as a captured HIP graph (below) */
} mhs_opts;

/* Dirichlet data on the faces other than the base.  Section 2.2 takes
 * B = 0 there, i.e. P = 0 on the side and top faces and on the edges of the
 * base (MHS_FACES_ZERO, the default); its procedure (summarised in Section
 * 5) leaves the other boundary conditions to the problem.  With
 * MHS_FACES_GIVEN the values already in P on those faces (the edges of
 * plane 0 for mhs_solve_boundary; the side and top faces for
 * mhs_solve_interior) are the Dirichlet data and are not modified.
 * mhs_fields still applies the B = 0 reading on the side and top faces, so
 * with given faces only its interior nodes are the fields of P. */
#define MHS_FACES_ZERO 0
#define MHS_FACES_GIVEN 1

typedef struct mhs_info {
    int32_t status;       /* MHS_OK or an MHS_ERR_* code                    */
    int32_t cycles;       /* V-cycles (FP64) / refinement steps (mixed)     */
    int32_t inner_cycles; /* total FP32 V-cycles (mixed path)               */
    int32_t host_syncs;   /* status read-backs performed                    */
    double rel_residual;  /* final ||r||_2 / ||r_0||_2                      */
    double r0;            /* ||r_0||_2                                      */
    double seconds;       /* wall time of the call                          */
} mhs_info;

typedef struct mhs_plan mhs_plan;

/* Fill *opts with defaults: FP64, V(2,2), rtol 1e-10, max_cycles 100,
 * inner_cycles 3, check_every 0 (adaptive), graph 0.
 *
 * opts->graph: the launches of one V-cycle (FP64) or refinement step
 * (mixed) of a solve are the same in every cycle of the call and, for a
 * plan, in every call with the same launch shapes; with graph = 1 they are
 * captured once as a HIP graph (kept by the plan, at most eight, on a
 * capture stream of its own) and replayed per cycle, with graph = 0
 * launched one by one.  Results are bitwise the same either way.  Off by
 * default: on MI355X the replays were 1-7 % slower than launching the
 * kernels (33^3 to 257^3, both paths).  Ignored (launched one by one) while
 * the plan profiles (mhs_profile_enable) and by mhs_solve_interior_noalloc. */
void mhs_default_opts(mhs_opts *opts);

/* Library version as 10000*major + 100*minor + patch. */
int32_t mhs_version(void);

/* Message describing the last failure on this thread ("" if none). */
const char *mhs_last_error(void);

/* Bytes of device workspace a plan for `grid` needs.  `precisions` is a
 * bit mask of MHS_PREC_* paths the plan must support (at least one), plus
 * MHS_PLAN_GENERAL for the general-operator entry points (about 3.4 more
 * doubles per node of the grid, and the same for its faces).  Validates the grid
 * (MHS_ERR_GRID for a bad axis). */
int mhs_workspace_bytes(const mhs_grid *grid, int32_t precisions, size_t *bytes);

/* Device memory one request of `grid` holds while it is served: the plan's
 * workspace (mhs_workspace_bytes for `precisions`) plus its arrays, bz0
 * (nx*ny doubles), P and the five field outputs (6*nx*ny*nz doubles).  The
 * batch counts this against its budget at admission (mhs_batch_create).
 * Errors: MHS_ERR_INVALID_ARG, MHS_ERR_GRID. */
int mhs_request_bytes(const mhs_grid *grid, int32_t precisions, size_t *bytes);

/* Host-only check of a model against a grid (no device work).  Every
 * interior plane must have xi < 1 (ellipticity of (8), Section 2.1) and
 * alpha^2 must lie below the smallest eigenvalue lambda_0 of
 * -[(1 - xi)(d2x + d2y) + d2z] on the grid, so that the discrete problem is
 * definite.  Coarse grids under-resolve the lowest mode, whose eigenvalue
 * lambda_l drops as the grid coarsens: the 3D hierarchy stops above the
 * first level with lambda_l - alpha^2 < (lambda_0 - alpha^2) / 2 (there the
 * coarse correction would over-correct that mode more than twofold) and
 * solves its parent exactly (at most 512 unknowns).  *lambda_min (optional)
 * receives lambda_0, *levels (optional) the number of 3D levels the solve
 * will use.  Returns MHS_OK, MHS_ERR_GRID, MHS_ERR_INVALID_ARG,
 * MHS_ERR_NOT_ELLIPTIC or MHS_ERR_INDEFINITE (alpha^2 >= lambda_0, or too
 * close to resonance for a coarse grid of at most 512 unknowns). */
int mhs_check_model(const mhs_grid *grid, const mhs_model *model, double *lambda_min, int32_t *levels);

/* Create a plan on the current HIP device over the caller's workspace
 * (d_workspace: device pointer, 256-byte aligned, >= mhs_workspace_bytes).
 * Clears the workspace (synchronously).  Each step of the 3D hierarchy
 * halves every axis, except that it keeps z when dz^2 >= 2 max(dx, dy)^2
 * (restriction and prolongation within planes) and keeps x and y when
 * 2 dz^2 <= min(dx, dy)^2 (restriction and prolongation along z); the 2D
 * hierarchy halves both axes.  Coarsening stops when an axis to be halved
 * has 3 nodes; the coarsest grid is solved exactly.  (The paper, Section
 * 2.2, leaves the coarse grids open; halving only the finer axes makes the
 * coarse levels equally spaced, which point smoothing needs.) */
int mhs_plan_create(const mhs_grid *grid, int32_t precisions, void *d_workspace,
                    size_t workspace_bytes, mhs_plan **plan);

/* Release the plan's host resources (not the caller's workspace). */
int mhs_plan_destroy(mhs_plan *plan);

/* Number of 3D (space = 3) or 2D (space = 2) multigrid levels of the plan,
 * and the node counts of level `level` (0 = finest). */
int mhs_plan_levels(const mhs_plan *plan, int32_t space, int32_t *nlevels);
int mhs_plan_level_dims(const mhs_plan *plan, int32_t space, int32_t level, int32_t *nx,
                        int32_t *ny, int32_t *nz);

/* First level (0 = finest) handled by the single-workgroup bottom solver,
 * which runs whole V-cycles from that level down to the coarsest grid. */
int mhs_plan_bottom_level(const mhs_plan *plan, int32_t space, int32_t *level);

/* Step 2 of the procedure of Section 2.2: multigrid solve of equation (11).
 * d_bz0: device, nx*ny doubles (edge values are not read).  d_P: device,
 * nx*ny*nz doubles; plane k = 0 (its first nx*ny doubles) receives P0 with
 * zero edges (or keeps the given edges, opts->faces); the other planes are
 * not touched.  Initial guess 0 unless
 * opts->warm_start.  Always FP64.  On MHS_ERR_NO_CONVERGENCE plane 0 holds
 * the last iterate and *info is filled. */
int mhs_solve_boundary(mhs_plan *plan, const double *d_bz0, double *d_P, const mhs_opts *opts,
                       mhs_info *info, void *stream);

/* Step 3 of the procedure: multigrid solve of equation (8) in place.  Plane
 * k = 0 of d_P is the Dirichlet data from mhs_solve_boundary; the side and
 * top faces are set to 0 (or kept as given, opts->faces); the interior
 * starts from 0 (step 1) unless
 * opts->warm_start.  opts->precision selects plain FP64 V-cycles or FP32
 * V-cycles inside FP64 iterative refinement (fine residual, update and the
 * coarsest solve in FP64).  Validates xi < 1 on interior planes
 * (MHS_ERR_NOT_ELLIPTIC) and definiteness (MHS_ERR_INDEFINITE) first. */
int mhs_solve_interior(mhs_plan *plan, const mhs_model *model, double *d_P, const mhs_opts *opts,
                       mhs_info *info, void *stream);

/* Field recovery (Section 2.2, equations (5), (6), (9), (10)) by central
 * differences: Bx = alpha P_y + P_xz, By = -alpha P_x + P_yz,
 * Bz = -(P_xx + P_yy), p = p_b - xi Bz^2/(2 mu0),
 * rho = rho_b + (xi' Bz^2/(2 mu0) + xi B.grad(Bz)/mu0)/g.
 * Faces: B = 0 on the side and top faces (so p = p_b, rho = rho_b there);
 * on the base the z-derivatives are one-sided second order.  All outputs
 * nx*ny*nz doubles on the device.  Asynchronous. */
int mhs_fields(mhs_plan *plan, const mhs_model *model, const double *d_P, double *d_Bx,
               double *d_By, double *d_Bz, double *d_p, double *d_rho, void *stream);

/* Steps 2 and 3 of the procedure and the field recovery in one call: the
 * same work and results (bitwise) as mhs_solve_boundary(opts2d), then
 * mhs_solve_interior(opts3d), then mhs_fields, on one stream, with fewer
 * host round trips: the model's 3D tables are computed on the host while
 * the base cycles run, and the field recovery is enqueued behind every
 * batch of interior cycles, running only once the solve has converged with
 * its iterate in d_P (else it runs after the final copy).  d_Bx ... d_rho:
 * all five (nx*ny*nz doubles on the device) or all NULL (no recovery).
 * Errors as the three calls; the first failing step ends the call (a base
 * solve that does not converge leaves the interior and the outputs
 * untouched).  Returns when the interior solve's status is known; the
 * recovery may still run on the stream. */
int mhs_solve_equilibrium(mhs_plan *plan, const mhs_model *model, const double *d_bz0, double *d_P,
                          double *d_Bx, double *d_By, double *d_Bz, double *d_p, double *d_rho,
                          const mhs_opts *opts2d, const mhs_opts *opts3d, mhs_info *info2d,
                          mhs_info *info3d, void *stream);

/* ---- the general elliptic problem (Section 2.2) -------------------------- *
 * Section 2.2 reduces the model to scalar problems of the form
 *     a(x) lap u + b(x) u = c(x) in D,  u given on the boundary of D,
 * with lap the 3D Laplacian in the interior or the 2D one on a boundary
 * face, and notes that elliptic problems other than (11) may be posed on
 * the other faces.  These entry points solve that form with per-node a, b,
 * c (second-order central differences, the plan's grid) by FP64 V(nu1,nu2)
 * multigrid: each interior row is divided by a (lap u + (b/a) u = c/a, the
 * same discrete solution; the residual and stopping rule are those of this
 * form), red-black Gauss-Seidel, the full weighting, interpolation and
 * coarsening of the solve of (8), b/a sampled at the coarse nodes, and an
 * exact solve of the coarsest grid (at most 96 unknowns, else
 * MHS_ERR_UNSUPPORTED).  The plan must have been created with
 * MHS_PLAN_GENERAL in its mask (else MHS_ERR_UNSUPPORTED);
 * opts->precision must be MHS_PREC_FP64; opts->faces is ignored (the
 * boundary values in u are always the data).  Errors before any cycle:
 * MHS_ERR_INVALID_ARG if a vanishes or a, b, c are not finite at an
 * interior node; MHS_ERR_INDEFINITE unless max(b/a) stays below half the
 * smallest eigenvalue of -lap on the coarsest grid (then every level is
 * definite and no coarse correction over-corrects the lowest mode).  The
 * call reads back once after that check and then like the other solves. */

/* 3D: d_a, d_b, d_c, d_u: device, nx*ny*nz doubles (x fastest).  u's
 * boundary nodes are the Dirichlet data (not modified); its interior
 * starts from 0 unless opts->warm_start and receives the solution. */
int mhs_solve_general(mhs_plan *plan, const double *d_a, const double *d_b, const double *d_c, double *d_u,
                      const mhs_opts *opts, mhs_info *info, void *stream);

/* A face of the box: the 2D problem on face `face` of d_P (nx*ny*nz
 * doubles), with the face's own edges (values in d_P) as Dirichlet data;
 * the interior nodes of that face of d_P receive the solution, nothing else
 * of d_P is written.  Face coordinates (first index fastest) and the shape
 * of d_a, d_b, d_c (device, contiguous):
 *   MHS_FACE_BASE (z = 0), MHS_FACE_TOP (z = lz): (x, y), ny*nx values;
 *   MHS_FACE_XLO (x = 0), MHS_FACE_XHI (x = lx): (y, z), nz*ny values;
 *   MHS_FACE_YLO (y = 0), MHS_FACE_YHI (y = ly): (x, z), nz*nx values.
 * Filling the side and top faces this way and then calling
 * mhs_solve_interior with opts->faces = MHS_FACES_GIVEN poses (8) with
 * boundary data from elliptic problems on every face. */
#define MHS_FACE_BASE 0
#define MHS_FACE_TOP 1
#define MHS_FACE_XLO 2
#define MHS_FACE_XHI 3
#define MHS_FACE_YLO 4
#define MHS_FACE_YHI 5
int mhs_solve_face(mhs_plan *plan, int32_t face, const double *d_a, const double *d_b, const double *d_c,
                   double *d_P, const mhs_opts *opts, mhs_info *info, void *stream);

/* ---- stage entry points (kernel-level checks; asynchronous) ----------- *
 * `space` is 3 (equation (8) at 3D level `level`) or 2 (equation (11) at
 * 2D level `level`); `precision` is MHS_PREC_FP64 (double arrays) or
 * MHS_PREC_MIXED (float arrays, the inner solver's storage).  Arrays have
 * the level's shape; boundary nodes of u are its Dirichlet values.  For
 * space 3 the model supplies xi and alpha; for space 2 it may be NULL.
 * The coarse coefficients use xi sampled at the coarse nodes.  These run
 * the same kernels as the solves. */

/* u <- nsweeps red-black Gauss-Seidel sweeps on A u = f (f may be NULL:
 * zero).  Red = (i+j+k) even, updated first.  zero_guess = 1: the first
 * sweep starts from u = 0 (the start of a coarse-grid correction, whose
 * Dirichlet data are zero): the interior values of u are not read, and its
 * boundary values, which later sweeps read, must be 0.  zero_guess must be
 * 0 or 1, and 1 needs f. */
int mhs_stage_smooth(mhs_plan *plan, const mhs_model *model, int32_t space, int32_t level,
                     int32_t precision, void *d_u, const void *d_f, int32_t nsweeps,
                     int32_t zero_guess, void *stream);

/* f_c <- full weighting of r = f - A u (r = 0 on boundary nodes) onto the
 * interior nodes of level+1; boundary nodes of f_c are not written. */
int mhs_stage_restrict(mhs_plan *plan, const mhs_model *model, int32_t space, int32_t level,
                       int32_t precision, const void *d_u, const void *d_f, void *d_fc,
                       void *stream);

/* u <- nsweeps (>= 1) red-black sweeps applied to u + I(e_c), where I is
 * trilinear (bilinear in 2D) interpolation from level+1, added on interior
 * nodes only (the first sweep fused with it, as in the cycle). */
int mhs_stage_correct_smooth(mhs_plan *plan, const mhs_model *model, int32_t space,
                             int32_t level, int32_t precision, void *d_u, const void *d_f,
                             const void *d_ec, int32_t nsweeps, void *stream);

/* u <- one V(nu1,nu2) cycle, starting from u = 0, on A u = f over the
 * plan's bottom levels (from level mhs_plan_bottom_level() to the coarsest,
 * which is solved exactly).  u and f must have the shape of that level;
 * *bottom_level (may be NULL) receives it.  Computed in FP64 whatever the
 * storage precision. */
int mhs_stage_bottom(mhs_plan *plan, const mhs_model *model, int32_t space, int32_t precision,
                     void *d_u, const void *d_f, int32_t nu1, int32_t nu2,
                     int32_t *bottom_level, void *stream);

/* *norm <- ||f - A u||_2 over interior nodes of the level (synchronous). */
int mhs_stage_residual_norm(mhs_plan *plan, const mhs_model *model, int32_t space,
                            int32_t level, int32_t precision, const void *d_u, const void *d_f,
                            double *norm, void *stream);

/* ---- diagnostics --------------------------------------------------------- *
 * Residuals of the MHS equations of Section 2.1 for fields on the plan's
 * grid (normally those of mhs_fields): j = (curl B)/mu0 from (2), the
 * magnitude of the force-balance residual |j x B - grad p - rho g e_z| of
 * (1), and div B of (3), each by second-order differences as in the field
 * recovery (central in x, y and above the base; one-sided second order,
 * (-3 f0 + 4 f1 - f2)/(2 dz), on the base plane k = 0).  On the side faces
 * and the top face, where the recovery sets B = 0, every output is 0.
 * A converged equilibrium gives fres and divb of the order of the
 * truncation error (O(h^2) relative to |j x B|).
 * All arrays are device (nz, ny, nx) FP64, x fastest, caller-owned; inputs
 * are read only; the ten arrays must not overlap.  model: only mu0 (> 0)
 * and g are read.  Asynchronous on `stream`; allocates nothing.
 * Errors: MHS_ERR_INVALID_ARG (NULL pointer, mu0 <= 0), MHS_ERR_HIP. */
int mhs_diagnostics(mhs_plan *plan, const mhs_model *model, const double *d_Bx, const double *d_By,
                    const double *d_Bz, const double *d_p, const double *d_rho, double *d_jx,
                    double *d_jy, double *d_jz, double *d_fres, double *d_divb, void *stream);

/* ---- field lines --------------------------------------------------------- *
 * Magnetic field lines, the curves through which Section 3 presents each
 * equilibrium (the paper does not say how it traces them).  Line l starts at
 * seed l and follows dx/ds = B/|B| in arc length s with the classical
 * fourth-order Runge-Kutta method and a fixed step ds (ds < 0 traces against
 * B).  B between nodes is the trilinear interpolation of the node values of
 * the cell holding the point (nested linear interpolations along x, then y,
 * then z); a Runge-Kutta stage outside the box takes the value at its
 * coordinates clamped to the box.  A line ends when a step would leave the
 * box [0, lx] x [0, ly] x [0, lz] (status 1; that point is dropped), when a
 * stage finds |B| <= bmin (status 2: a null), or after max_steps steps
 * (status 0); a seed outside the box gives a line of one point, status 1.
 * d_Bx, d_By, d_Bz: device (nz, ny, nx) FP64 on the plan's grid (normally
 * from mhs_fields).  d_seeds: device nlines x 3 (x, y, z).  d_points: device
 * (max_steps + 1) x nlines x 3, point n of line l at 3 (n nlines + l)
 * (point 0 = the seed; points past d_count[l] are not written).  d_count,
 * d_status: device int32, nlines each.  All caller-owned; asynchronous on
 * `stream`; allocates nothing.  Errors: MHS_ERR_INVALID_ARG (NULL pointer
 * with nlines > 0, nlines < 0, max_steps < 0, ds zero or not finite, bmin
 * negative or not finite), MHS_ERR_HIP. */
#define MHS_LINE_MAX_STEPS 0
#define MHS_LINE_EXIT 1
#define MHS_LINE_NULL 2
int mhs_trace_field_lines(mhs_plan *plan, const double *d_Bx, const double *d_By, const double *d_Bz,
                          const double *d_seeds, int32_t nlines, double ds, int32_t max_steps, double bmin,
                          double *d_points, int32_t *d_count, int32_t *d_status, void *stream);

/* ---- measurement ------------------------------------------------------- *
 * When profiling is enabled on a plan, each launch of the selected kernel
 * classes below is bracketed by HIP events on the call's stream (select
 * few classes to keep the perturbation small: each event is a queue
 * packet between kernels).  Solves count only
 * cycles that executed (the status read-back tells how many), so launches
 * skipped by the device-side stopping flag are excluded.  Each launch also
 * adds its compulsory HBM traffic (bytes the kernel must read and write:
 * each input array once, each output once) to the class. */
#define MHS_PROF_SMOOTH_L0 0   /* finest-level 3D smoother, FP64 or FP32  */
#define MHS_PROF_REFINE 1      /* FP64 refinement update + residual       */
#define MHS_PROF_RESTRICT_L0 2 /* finest-level residual + restriction     */
#define MHS_PROF_FIELDS 3      /* field recovery                          */
#define MHS_PROF_BOTTOM 4      /* single-workgroup bottom solver          */
#define MHS_PROF_COARSE 5      /* every other stencil launch (levels >= 1, 2D, z-only prolongation) */
#define MHS_PROF_DIAG 6        /* diagnostics (mhs_diagnostics)            */
#define MHS_PROF_TRACE 7       /* field lines (mhs_trace_field_lines)      */
#define MHS_PROF_GENERAL 8     /* general operator (mhs_solve_general, _face) */
#define MHS_PROF_NCLASS 9
#define MHS_PROF_ALL 0x1ff     /* mask of every class                      */

/* class_mask: bit (1 << MHS_PROF_x) times class x; 0 disables profiling. */
int mhs_profile_enable(mhs_plan *plan, int32_t class_mask);
/* Totals since the last reset for one class (synchronizes pending events). */
int mhs_profile_read(mhs_plan *plan, int32_t klass, double *total_ms, int64_t *launches,
                     double *bytes, int32_t reset);

/* ---- continuous batching (serving) ------------------------------------ *
 * A batch advances many independent equilibria together.  Each admitted
 * request goes through the procedure of Section 2.2: the lower-boundary
 * solve of (11), the interior solve of (8) (FP64 V-cycles or FP32-in-FP64
 * refinement), then the field recovery.  One tick advances every active
 * slot by one V-cycle (or one refinement step) of its current phase; the
 * launches of a tick are merged across slots, so each stage of the tick is
 * one descriptor-driven launch covering every slot that has it (requests
 * of different shapes and precisions share launches).  The merged path
 * runs the same kernels with the same per-request tiling and reduction
 * order as the single-request entry points, so a request gives bit-for-bit
 * the result of mhs_solve_boundary + mhs_solve_interior + mhs_fields.
 *
 * Memory: the batch holds per-slot status words and its launch-descriptor
 * tables in a caller-provided device workspace of
 * mhs_batch_workspace_bytes(max_slots) bytes (256-byte aligned); each slot
 * uses its own plan's workspace for everything else.  Admission by HBM
 * footprint: a batch created with an hbm_budget admits a request only while
 * the footprints (mhs_request_bytes) of the requests it holds, this one
 * included, stay within that budget; a request holds its footprint from
 * admission until mhs_batch_release.  The batch allocates none of that
 * memory (the caller does, before admission); queueing requests that do
 * not fit and pooling plans between requests belong to the caller.
 * A batch is used from one host thread.  Ticks are pipelined two deep:
 * mhs_batch_step launches tick t and then reads the status of tick t-1
 * while the device works on tick t, so a request's completion is seen one
 * call after the tick that completed it, and a request that stopped in
 * tick t-1 had one more cycle launched in tick t whose kernels exit at
 * once on its status word (results are unchanged). */
typedef struct mhs_batch mhs_batch;

/* Device workspace a batch of max_slots (1..1024) slots needs. */
int mhs_batch_workspace_bytes(int32_t max_slots, size_t *bytes);

/* Create a batch on the current device over d_ws (owned by the caller,
 * kept until mhs_batch_destroy).  hbm_budget: bytes of device memory the
 * admitted requests may hold together (0 = no limit; see Memory above).
 * Allocates host structures and pinned status/descriptor buffers only. */
int mhs_batch_create(int32_t max_slots, size_t hbm_budget, void *d_ws, size_t ws_bytes, mhs_batch **batch);
int mhs_batch_destroy(mhs_batch *batch);

/* Footprint (mhs_request_bytes) of the requests the batch holds now. */
int mhs_batch_bytes_in_use(const mhs_batch *batch, size_t *bytes);

/* Admit one request into a free slot.  The plan must be exclusive to this
 * slot until the slot is released (a plan already held by an active slot
 * gives MHS_ERR_INVALID_ARG) and live on the batch's device.  d_bz0
 * ((ny, nx)), d_P and the five field outputs ((nz, ny, nx)) must stay valid
 * until the slot is released.  Model arrays are copied; the model's
 * coefficient tables and the coarsest-grid inverse are built here
 * (synchronously), so admission can fail with MHS_ERR_NOT_ELLIPTIC or
 * MHS_ERR_INDEFINITE.  opts->precision selects the interior path (the
 * boundary solve is always FP64); opts->rtol and max_cycles apply to both
 * solves; opts->check_every is ignored (every tick reads the status).
 * MHS_ERR_BUDGET: no free slot, the request's footprint would take the
 * batch over its hbm_budget, or the request's per-tick descriptors exceed
 * the slot's share of the descriptor table (very large nu1, nu2 or
 * inner_cycles).  On success *slot is the slot index (0..max_slots-1). */
int mhs_batch_admit(mhs_batch *batch, mhs_plan *plan, const mhs_model *model,
                    const double *d_bz0, double *d_P, double *d_Bx, double *d_By, double *d_Bz,
                    double *d_p, double *d_rho, const mhs_opts *opts, int32_t *slot);

/* Launch one tick on `stream`, then wait for the previous tick and apply
 * its status (phase changes, completions).  *active (optional) receives the
 * number of slots still running; call until it is 0.  Use one stream for
 * every call of a batch (and for the copies into its requests' buffers). */
int mhs_batch_step(mhs_batch *batch, void *stream, int32_t *active);

/* Status of a slot.  *done = 1 once the request has finished: its fields
 * are written (status MHS_OK) or one of its solves stopped with an error
 * (the slot's info carries the code; later phases are not run).
 * `boundary` and `interior` (optional) receive the per-solve info: cycles,
 * refinement steps, residuals, status; `seconds` is the wall time from
 * admission to the end of that phase. */
int mhs_batch_poll(mhs_batch *batch, int32_t slot, int32_t *done, mhs_info *boundary,
                   mhs_info *interior);

/* Free a slot (finished or not) for reuse; its plan may then be reused. */
int mhs_batch_release(mhs_batch *batch, int32_t slot);

/* Profiling of a batch's merged launches (the MHS_PROF_* classes above):
 * each launch of a selected class is bracketed by HIP events on the tick's
 * stream.  A merged launch counts once if any of its requests' items ran
 * (items after a request's convergence check exit at once in the tick the
 * request stops); its compulsory bytes are the sum over the items that
 * ran.  class_mask 0 disables; bits outside MHS_PROF_ALL are
 * MHS_ERR_INVALID_ARG.  profile_read returns the totals since the last
 * reset over the ticks whose status has been read. */
int mhs_batch_profile_enable(mhs_batch *batch, int32_t class_mask);
int mhs_batch_profile_read(mhs_batch *batch, int32_t klass, double *total_ms, int64_t *launches,
                           double *bytes, int32_t reset);

/* ---- access-pattern reference (a measurement aid, not part of a solve) -- *
 * Moves the compulsory bytes of a level-0 FP32 smoother launch (read u_in
 * and f, write u_out: 12 bytes per interior node) in the smoother's memory
 * order, with no LDS, barrier or arithmetic worth the name, so that its
 * rate is the ceiling the z-marching tile pattern itself allows: per
 * workgroup an x-y tile of interior nodes of one request marching kz planes
 * (from two planes below the chunk to one above it), reading the tile plus
 * a two-node ring of every plane of u_in two planes ahead of use, f at the
 * tile's nodes of the chunk's planes, and writing u_out at those nodes.
 * d_u, d_f, d_out: nreq device arrays of nx*ny*nz floats each, x-fastest,
 * request r at element offset r*nx*ny*nz (caller-owned, distinct).  tile 0
 * is the smoother's tile (64 x 16 nodes, 512 threads), tile 1 a row-wide
 * tile (256 x 8 nodes, 1024 threads); kz >= 1.  Overwrites the interior
 * nodes of d_out with f plus 1e-30 times a sum of loaded values (finite
 * inputs stay finite) and nothing else.  Asynchronous on `stream`.  Errors:
 * MHS_ERR_INVALID_ARG for NULL pointers, nx, ny or nz < 3, nreq or kz < 1,
 * another tile; MHS_ERR_HIP if the launch fails. */
int mhs_probe_smoother_pattern(const float *d_u, const float *d_f, float *d_out, int32_t nx, int32_t ny,
                               int32_t nz, int32_t nreq, int32_t tile, int32_t kz, void *stream);

/* ---- interior solve without allocation -------------------------------- *
 * For callers that cannot allocate device memory or create a plan (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): mhs_solve_interior for `grid` without a plan or workspace.
 * Same arguments, semantics, kernels and results as mhs_solve_interior on a
 * plan of the same grid (bitwise), with opts->precision selecting the path.
 * The hierarchy lives in a fixed device array of 48 MiB inside the library
 * (one copy per device, held until the process ends), so the grid's
 * workspace for that one precision must fit: grids up to 129 x 129 x 129
 * with either precision; larger ones return MHS_ERR_WORKSPACE before any
 * device work.  Devices 0..15 (else MHS_ERR_UNSUPPORTED).  The call
 * allocates no device or pinned host memory (host bookkeeping uses the C++
 * heap), clears the part of the array it uses with a fill kernel, and
 * returns once its stream has drained.  Every call on a device shares that
 * device's array and finds the previous call's contents in it: calls on one
 * device from several threads of a process are serialised by the library;
 * work of another library instance or a caller's kernel that touched the
 * array concurrently would race with it. */
int mhs_solve_interior_noalloc(const mhs_grid *grid, const mhs_model *model, double *d_P,
                               const mhs_opts *opts, mhs_info *info, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MHS_H */
