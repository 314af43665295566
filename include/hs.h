/*
 * hs.h -- C ABI of the MI355X (gfx950) implementation of the per-time-step particle update
 * of the hybrid stochastic-particle-Shakhov / DSMC method (Jin, Liu, Yang, Cao, Zhuo,
 * Zhong, arXiv 2506.23917, Sec. 3).
 *
 * One step, on the GPU, for a batch of independent flow cases sharing one particle array:
 *   inflow injection -> free transport with walls (Step 2, Eq. 4, Eq. 30) -> stable cell
 *   counting sort (Step 3) -> per cell: moments (Eq. 31), time split (Eq. 25-28), NTC DSMC
 *   (Eq. 5-9), SP-Shakhov resampling (Eq. 16-18), conservation rescale (Eq. 19),
 *   time-averaged sampling (Step 5).
 *
 * Conventions
 *  - SI units.  Cells of a grid case are numbered x-fastest, cell c = i + nx (j + ny k);
 *    cells of a mesh case as in its hs_mesh.
 *  - Memory: the CALLER owns all device memory.  hs_plan() gives the workspace size; the
 *    caller allocates it (e.g. a torch uint8 tensor on the GPU) and passes it to
 *    hs_init_particles(), which carves every buffer out of it.  The workspace must
 *    outlive the sim.  The sim handle owns host metadata only.
 *  - Streams: all GPU work of a sim is enqueued on the hipStream_t given at init
 *    (passed as void*; NULL = the default stream).  hs_step() does not synchronise.
 *    Within a step the dense-cell kernel runs on a second stream that the sim creates
 *    (default priority, non-blocking) and destroys: it is forked from the given stream
 *    after the scatter and joined back into it before the step ends, so work queued later on
 *    the given stream, or a graph captured from it, sees the whole step.  Calls that
 *    return data (hs_sample_moments, hs_export_state, hs_last_trace, hs_counters, hs_sync)
 *    synchronise the given stream.
 *  - Errors: every call returns an hs_status.  Argument errors return at once and
 *    change nothing.  Faults found on the device (capacity overflow, a non-finite
 *    moment, inconsistent state) are latched in a device error word and reported by the
 *    next synchronising call; after that the sim answers HS_ERR_STATE to everything but
 *    hs_error_string/hs_destroy.  A cell may hold any number of particles up to the
 *    case's capacity (cells above 4096 particles are worked on in device memory instead
 *    of LDS, more slowly).
 *  - Not thread-safe: one sim, one host thread, one stream.
 *  - Randomness: Philox4x32-10 keyed by each case's seed; counters are
 *    (entity, stream, step, draw) with entities local to the case, so a case gives the
 *    same result alone or in any batch.  Seeds must differ between cases of a batch.
 */
#ifndef HS_H
#define HS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HS_OK = 0,
    HS_ERR_ARG = 1,        /* invalid argument                                        */
    HS_ERR_CAPACITY = 2,   /* particle capacity (or a static-scratch size) exceeded   */
    HS_ERR_NUMERIC = 3,    /* non-finite velocity or moment                           */
    HS_ERR_DEVICE = 4,     /* a HIP runtime call failed                               */
    HS_ERR_STATE = 5       /* the sim is in a failed state                            */
} hs_status;

typedef enum { HS_FP64 = 0, HS_FP32_MIXED = 1 } hs_precision;
typedef enum { HS_BC_OUTFLOW = 0, HS_BC_SPECULAR = 1, HS_BC_INFLOW = 2 } hs_bc;
typedef enum { HS_BODY_NONE = 0, HS_BODY_CYLINDER = 1, HS_BODY_SPHERE = 2 } hs_body;
/* What lies across a mesh edge that has no neighbour cell (see hs_mesh). */
typedef enum {
    HS_EDGE_OUTFLOW = -1, HS_EDGE_INFLOW = -2, HS_EDGE_WALL = -3, HS_EDGE_SPECULAR = -4
} hs_edge;

enum {
    HS_FLAG_TRACE = 1,         /* keep a per-cell record of the last step (hs_last_trace)  */
    HS_FLAG_NO_PARTICLES = 2,  /* hs_init_particles leaves the domain empty (for import)    */
    HS_FLAG_GRAPH = 4,         /* replay each step as a captured hipGraph                   */
    HS_FLAG_STATIC_SCRATCH = 8 /* hs_plan only: size the data part for hs_init_particles_static */
};

/* Size of the library's fixed device scratch array used by hs_init_particles_static. */
#define HS_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)

/* Kernel groups of one step, for hs_kernel_timing (bit k of the timing mask = group k). */
enum {
    HS_KERNEL_INJECT = 0,      /* inflow counts, scan and fill (Step 2 freestream faces)     */
    HS_KERNEL_MOVE = 1,        /* free transport, walls, per-cell counts (Step 2)           */
    HS_KERNEL_SCAN = 2,        /* exclusive scan of the cell counts, tile table             */
    HS_KERNEL_SCATTER = 3,     /* scatter of particle indices by cell                       */
    HS_KERNEL_GATHER = 4,      /* stable in-cell order, sorted state written                */
    HS_KERNEL_SCALARS = 5,     /* Step 3 moments, Eq. 10 / 25-28 split, N_col per cell      */
    HS_KERNEL_COLLIDE = 6,     /* Step 4-5 on the tiles: NTC, Shakhov, rescale, sampling    */
    HS_KERNEL_DENSE = 7,       /* Steps 3-5 of the cells too dense for the tiles            */
    HS_KERNEL_STEP = 8,        /* the whole step                                            */
    HS_NUM_KERNELS = 9
};

/* Gas (Sec. 4): molecular mass, VHS reference diameter / temperature / viscosity and
 * exponent omega, Prandtl number (Shakhov model, Eq. 12), specific-heat ratio (Eq. 25). */
typedef struct {
    double m, d_ref, T_ref, omega, mu_ref, Pr, gamma;
} hs_gas;

/* Drifting Maxwellian: number density (1/m^3), velocity (m/s), temperature (K). */
typedef struct {
    double n, u[3], T;
} hs_state;

/* A body-fitted mesh, the paper's unstructured meshes (Sec. 4.2 the cylinder's O-grid,
 * Sec. 4.3 the jet's quads, Sec. 4.4 the sphere's hexahedra), tracked face to face.
 *  2-D (case dim 2), convex quadrilaterals: xy has 2 doubles per node (m); quad 4 node ids
 *    per cell, counter-clockwise; nbr 4 per cell, entry j across edge j (node j -> node
 *    (j+1) mod 4).
 *  3-D (case dim 3), convex hexahedra with planar faces (a face may collapse to a triangle
 *    or, never crossed, to a segment): xy has 3 doubles per node; quad 8 node ids per cell,
 *    0-3 the bottom face counter-clockwise seen from above and 4-7 above them; nbr 6 per
 *    cell, entry f across face f with nodes (0,3,2,1), (4,5,6,7), (0,1,5,4), (1,2,6,5),
 *    (2,3,7,6), (3,0,4,7).
 *  Across an edge or face: the neighbour cell, which must name this cell back across the
 *    same nodes, or an hs_edge code: OUTFLOW removes particles that cross it; INFLOW removes
 *    them and feeds the case's inflow state's one-way flux through it; WALL re-emits them
 *    diffusely at body_T about its normal; SPECULAR mirrors them.
 * Arrays are host memory, read and copied at init (the caller keeps ownership). */
typedef struct {
    int32_t n_nodes, n_cells;
    const double *xy;
    const int32_t *quad;
    const int32_t *nbr;
} hs_mesh;

/* One flow case on a uniform Cartesian grid or (mesh != NULL) on a quad mesh.
 *  dim 1..3: cells nx (x ny (x nz)); lo = lower corner, h = cell edges; for unused axes
 *    h is the unit depth/area, so every cell volume is h0 h1 h2 times its fluid fraction.
 *  dim 0: nx independent homogeneous cells (no transport), each with its own step
 *    dt_over_tau[k] * tau_0, tau_0 = mu(T) / (n k T) of region_state[0].
 *  bc: faces -x,+x,-y,+y,-z,+z.  OUTFLOW removes leaving particles; SPECULAR reflects;
 *    INFLOW removes leaving particles and injects the inflow state's one-way flux
 *    (only through faces whose centre lies inside [slot_lo, slot_hi) on every tangential
 *    axis with slot_hi > slot_lo).
 *  body: a diffusely reflecting cylinder (axis z) or sphere at T body_T, strictly inside
 *    the domain; cells are cut by it (fluid fraction = share of 16^dim sub-cell centres
 *    outside).  SPECULAR walls cannot be combined with a body.
 *  regions: initial state; a cell takes the state of the first box holding its centre
 *    (6 doubles per box: lo xyz, hi xyz); cells in no box start empty.
 *  F_N: real molecules per particle; dt_G: global time step (fixed; Eq. 26 evaluated by
 *    the caller); T_sigma: temperature setting the initial (sigma_T c_r)_max at
 *    c* = 10 sqrt(k T_sigma / m); n_steady: first sampled step (Step 5); capacity: the
 *    largest number of particles the case may hold.  Arrays are copied at init.
 *  n_surf: number of body surface elements sampled from step n_steady on (0: none; needs
 *    a body; at most 65536); see hs_surface_sample.
 *  adapt_dt: 0 keeps dt_G; 1 makes the global step adaptive (Eq. 26): the step after
 *    step s is the minimum over the case's active cells (N >= 2, T > 0) of the Eq. 25
 *    local step from step s's Step (3) moments, the first step uses dt_G, a step without
 *    active cells keeps the last value, and inflow counts scale with the step (dim >= 1;
 *    see hs_step_dt).
 *  mesh: NULL for the grid; else the cells are the mesh's quads (dim 2; volume = area x h[2],
 *    h[2] the depth; Eq. 25's L_cell = area / longest edge) or hexahedra (dim 3; L_cell =
 *    volume / largest face area), numbered as in the mesh; nx, ny, nz, lo, the in-plane h,
 *    bc and the slot are ignored; regions select cells by the mean of their nodes; body may
 *    be NONE or CYLINDER (2-D) / SPHERE (3-D) and only frames the surface elements
 *    (polar-angle bands about the WALL edges' or faces' normals; body_r sets the element
 *    areas and A_ref), the wall itself being the WALL edges or faces at body_T. */
typedef struct {
    int32_t dim, nx, ny, nz;
    double lo[3], h[3];
    int32_t bc[6];
    hs_state inflow;
    double slot_lo[3], slot_hi[3];
    int32_t body;
    double body_c[3], body_r, body_T;
    int32_t n_regions;
    const double *region_box;
    const hs_state *region_state;
    double F_N, dt_G, T_sigma;
    const double *dt_over_tau;
    uint64_t seed;
    int64_t n_steady, capacity;
    int32_t n_surf;
    int32_t adapt_dt;
    const hs_mesh *mesh;
} hs_case;

typedef struct hs_sim hs_sim;

/* Per-cell record of the last step (with HS_FLAG_TRACE): particle count, NTC candidates,
 * accepted pairs, relaxed particles, Shakhov attempts and capped draws, an
 * order-independent hash of the accepted candidate indices, the cell's T, tau,
 * DSMC sub-step, relaxation probability, Shakhov envelope, and sum c, sum |c|^2 before
 * the collision stage and after the rescale (FP64, before any rounding to FP32). */
typedef struct {
    int64_t n, ncol, nacc, nrelax, ar_attempts, ar_cap;
    uint64_t acc_hash;
    double T, tau, dt_dsmc, p_relax, a_max;
    double pre_sum[4];
    double post_sum[4];
} hs_trace;

/* Cumulative per-case event counters, in this order. */
enum {
    HS_CNT_INJECTED = 0, HS_CNT_REMOVED, HS_CNT_WALL_HITS, HS_CNT_CANDIDATES,
    HS_CNT_ACCEPTED, HS_CNT_RELAXED, HS_CNT_AR_ATTEMPTS, HS_CNT_AR_CAP,
    HS_CNT_BOUNCE_CAP, HS_CNT_INJECT_CAP, HS_CNT_SKIPPED_CELLS, HS_NUM_COUNTERS
};

/* Size in bytes of the device workspace for this batch (no GPU work).  With
 * HS_FLAG_STATIC_SCRATCH in flags: the size of the data part that hs_init_particles_static
 * takes, and HS_ERR_CAPACITY when the batch's scratch part exceeds HS_STATIC_SCRATCH_BYTES. */
hs_status hs_plan(const hs_gas *gas, const hs_case *cases, int n_cases, hs_precision prec,
                  uint32_t flags, size_t *dev_bytes);

/* Step (1), Sec. 3.2: validate and copy the cases, lay out the workspace, compute cut-cell
 * volumes, draw the initial particles (uniform positions in each cell's fluid part,
 * velocities U + Eq. 17 Maxwellian, N = floor(n V / F_N + u) per cell, ids in cell order)
 * and set (sigma_T c_r)_max.  dev_workspace: device pointer to >= hs_plan() bytes, owned
 * by the caller.  hip_stream: the hipStream_t to use.  On success *out is a new sim. */
hs_status hs_init_particles(const hs_gas *gas, const hs_case *cases, int n_cases,
                            hs_precision prec, uint32_t flags, void *dev_workspace,
                            size_t dev_bytes, void *hip_stream, hs_sim **out);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): hs_init_particles with the step's scratch arrays
 * (new cells, slots, sort permutation, scan partials, tile tables, cell records, output
 * staging) placed in a fixed array inside the library, HS_STATIC_SCRATCH_BYTES on each device,
 * held until the process ends.  The caller passes only the sim's data part, dev_data of
 * data_bytes >= the size hs_plan reports with HS_FLAG_STATIC_SCRATCH (case tables, particle
 * state, per-cell state and sums, wall sums, trace records), which it owns as with
 * hs_init_particles.  The call allocates no device memory and creates no stream or event:
 * the sim's block-per-cell kernel runs on hip_stream before the tile kernels instead of on a
 * second stream.  Results are bit-identical to a sim made by hs_init_particles.
 * All such sims on one device share the one array and its contents: only one may exist per
 * device at a time (a second would overwrite the first's scratch; steps of two such sims that
 * overlap race).  Every scratch array is written before it is read in each step, so the
 * previous sim's contents need no clearing.  Errors: as hs_init_particles, plus
 * HS_ERR_CAPACITY when the batch's scratch exceeds HS_STATIC_SCRATCH_BYTES (*out is then
 * NULL) and HS_ERR_DEVICE when the array's device address cannot be found. */
hs_status hs_init_particles_static(const hs_gas *gas, const hs_case *cases, int n_cases,
                                   hs_precision prec, uint32_t flags, void *dev_data,
                                   size_t data_bytes, void *hip_stream, hs_sim **out);

/* Steps (2)-(5), n times, enqueued asynchronously on the sim's stream. */
hs_status hs_step(hs_sim *sim, int64_t n);

/* Block until the sim's stream is idle; report latched device errors. */
hs_status hs_sync(hs_sim *sim);

/* Step (6): per-cell output for case_id into caller-owned host arrays of ncells entries
 * (u3, q3: 3 per cell).  mode 0: time averages of the Step (5) sums since n_steady;
 * mode 1: the Eq. 31 estimators of the current particles.  Any pointer may be NULL. */
hs_status hs_sample_moments(hs_sim *sim, int case_id, int mode, double *n, double *u3,
                            double *T, double *q3, int64_t *n_samples);

/* Checkpoint of one case (native precision, bit-exact resume).  Layout: hs_state_header
 * (version 2; only that version is accepted),
 * then pos[3][np], vel[3][np] (element size 8 for HS_FP64, 4 for HS_FP32_MIXED; pos is
 * the cell-relative position in [0,1) per axis; on a mesh, the position relative to the
 * cell's first node, in m), cell[np] (int32, case-local),
 * id[np] (int64), sigc_max[ncells], acc[ncells][13] (double).  Particles are sorted by
 * cell.  hs_state_bytes gives the size.  Importing requires cells non-decreasing and every
 * id in [next_id - 2^32 + 1, next_id) (the device keeps an id's low 32 bits and restores it
 * from the case's next id, so a live particle's id is one of its case's last 2^32 ids; a
 * particle that stayed while 2^32 later particles entered its case would lose its id);
 * it sets the sim's step counter (shared by all cases); HS_ERR_ARG otherwise. */
typedef struct {
    uint32_t magic, version, precision, dim;
    int64_t np, ncells, next_id, step, n_samples;
    double dt_next, t_sampled;     /* the case's next global step and sampled time (v2) */
} hs_state_header;
size_t hs_state_bytes(hs_sim *sim, int case_id);
hs_status hs_export_state(hs_sim *sim, int case_id, void *host_buf, size_t bytes);
hs_status hs_import_state(hs_sim *sim, int case_id, const void *host_buf, size_t bytes);

/* Per-cell records of the last step (needs HS_FLAG_TRACE); out has ncells entries. */
hs_status hs_last_trace(hs_sim *sim, int case_id, hs_trace *out);

/* Cumulative counters of case_id, HS_NUM_COUNTERS int64 values. */
hs_status hs_counters(hs_sim *sim, int case_id, int64_t *out);

/* Number of cells / live particles of a case (the latter synchronises). */
int64_t hs_num_cells(const hs_sim *sim, int case_id);
int64_t hs_num_particles(hs_sim *sim, int case_id);

/* Per-kernel timing with HIP events recorded on the sim's stream around the kernel groups
 * selected by `mask` (bit k = HS_KERNEL_k; 0 turns timing off) in every step enqueued while
 * timing is on (steps then run as plain launches, not as a graph).  hs_kernel_timing
 * synchronises and returns the average duration (ms) of kernel group `which` over the
 * timed steps and their number (0 if the group was not selected); hs_clear_timing forgets
 * them.  hs_set_timing_period(sim, k) records the events in every k-th step of hs_step only
 * (counted from the last hs_clear_timing; k = 1, the default, times every step): the events
 * cost the stream a few microseconds each, so a long timed run samples its launches evenly
 * instead; HS_ERR_ARG for k < 1.  The autotuner times every step of its trials. */
hs_status hs_set_timing(hs_sim *sim, uint32_t mask);
hs_status hs_set_timing_period(hs_sim *sim, int period);
hs_status hs_kernel_timing(hs_sim *sim, int which, double *avg_ms, int64_t *launches);
hs_status hs_clear_timing(hs_sim *sim);

/* Launch-shape autotuner.  For each tunable kernel group (collide, gather, scalars, dense,
 * move, scatter) it runs `steps_per_trial` steps with each candidate grid size (blocks per
 * launch), timed with HIP events, and keeps the fastest; `report` (may be NULL) receives
 * the chosen grids, their average durations (ms) and the number of steps taken.  Grid
 * sizes do not change results -- every tile, cell and particle is processed the same way
 * whichever block takes it -- so the tuning steps are ordinary steps of the run: the
 * simulation advances by `report->steps`.  Synchronises; forgets timing records; a
 * captured step graph is dropped and captured again with the new shapes.  Errors: as
 * hs_step plus the device checks of hs_sync. */
typedef struct {
    int32_t grid[HS_NUM_KERNELS];   /* chosen blocks per launch (0: group not tuned)    */
    double ms[HS_NUM_KERNELS];      /* average duration of the chosen shape, ms         */
    int64_t steps;                  /* steps the tuning advanced the simulation         */
} hs_tune_report;
hs_status hs_autotune(hs_sim *sim, int steps_per_trial, hs_tune_report *report);

/* Set the grid size (blocks per launch) of kernel group `which` by hand; 0 restores the
 * built-in default.  Results do not depend on it.  Drops a captured step graph. */
hs_status hs_set_grid(hs_sim *sim, int which, int32_t blocks);

/* Body surface sampling: the wall counterpart of Step (5), giving the quantities of Eq. 35
 * (surface pressure and heat flux, with the shear stress the paper's surface plots show)
 * and Eq. 36 (drag and lift coefficients).  Element k of the case's n_surf elements holds
 * the wall points whose polar angle from the upstream stagnation direction -x lies in
 * [k, k+1) pi / n_surf (a cylinder's upper and lower halves together).  Every diffuse
 * reflection at the body during a sampled step (step >= n_steady) adds to its element:
 * 1, dP.n, dP.t, dE and dP (x, y, z), with dP = m F_N (c_in - c_out) the momentum given to
 * the wall, dE = m F_N (|c_in|^2 - |c_out|^2) / 2 the energy, n the outward normal and t
 * the unit tangent of growing polar angle at the hit point.  On a mesh, the wall points are
 * the WALL edges and n is the unit normal of the edge hit (pointing into the gas); its polar
 * angle chooses the element.
 *
 * hs_surface_sums copies these raw sums of case_id, n_surf x 7 doubles, into host memory.
 * hs_surface_sample gives their time averages over the S sampled steps of length dt_G:
 * per element 8 doubles (mid angle, area A, p = -sum dP.n / (A S dt_G),
 * tau = sum dP.t / (A S dt_G), q = sum dE / (A S dt_G), C_p = (p - p_inf) / (rho U^2 / 2),
 * C_f = tau / (rho U^2 / 2), C_h = q / (rho U^3 / 2)), and 5 doubles for the body (force
 * x, y, z = sum dP / (S dt_G); C_D and C_L = the force along u / |u| and along
 * (-u_y, u_x, 0) / |u| over rho U^2 A_ref / 2).  The freestream is the case's inflow
 * state (rho = n m, U = |u|, p_inf = n k T); coefficients are 0 when it has no speed.
 * Areas: a cylinder's element is its two strips, 2 R dtheta times the axial length (h_z in
 * 2-D, nz h_z in 3-D), with A_ref = 2 R times that length; a sphere's element is the zone
 * 2 pi R^2 (cos theta_k - cos theta_k+1), A_ref = pi R^2.  Outputs are caller-owned host
 * arrays (n_samples may be NULL).  Both synchronise the sim's stream.  Errors: HS_ERR_ARG
 * for a bad case_id, a case without surface elements or a NULL array; device errors as
 * hs_sync. */
hs_status hs_surface_sums(hs_sim *sim, int case_id, double *sums7);
hs_status hs_surface_sample(hs_sim *sim, int case_id, double *elem8, double *body5, int64_t *n_samples);

/* Global step of case_id that the next hs_step will use (dt_G, or the Eq. 26 value with
 * adapt_dt), and the sampled time (the sum of the global steps of the sampled steps).
 * Either pointer may be NULL.  Synchronises.  Errors: HS_ERR_ARG for a bad case_id. */
hs_status hs_step_dt(hs_sim *sim, int case_id, double *dt_next, double *t_sampled);

/* "Ratio of DSMC" of each cell of case_id, from the time-averaged moments of Step (6)
 * (n, U, T as hs_sample_moments mode 0): Dt_DSMC / Dt_G of Eq. 27, i.e. 1 where
 * Dt_c <= tau and tau / Dt_c elsewhere, with tau = mu(T) / (n k T) (Eq. 10) and Dt_c the
 * Eq. 25 local step (a 0-D cell: its own step); 0 for a cell without samples.  ratio is a
 * caller-owned host array of ncells doubles.  Synchronises.  Errors: HS_ERR_ARG for a bad
 * case_id or NULL array; device errors as hs_sync. */
hs_status hs_dsmc_ratio(hs_sim *sim, int case_id, double *ratio);

/* Human-readable description of the last error (never NULL). */
const char *hs_error_string(const hs_sim *sim);

/* Release host metadata (the workspace stays the caller's). */
void hs_destroy(hs_sim *sim);

/* Philox4x32-10 words for counters (entity, stream, step, draw) of one seed, computed on
 * the GPU into a caller-owned device array of 4 * n uint32 (entity = first_entity + i);
 * synchronous.  For cross-checking the generator. */
hs_status hs_debug_philox(uint64_t seed, uint32_t stream, uint64_t first_entity,
                          uint32_t step, uint32_t draw, int64_t n, void *dev_out,
                          void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
