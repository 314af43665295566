/*
 * hs_oracle.h -- plain FP64 CPU oracle of the per-time-step particle update of the
 * hybrid stochastic-particle-Shakhov / DSMC method (Jin et al., arXiv 2506.23917).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct reference the
 * GPU path is checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product library never does.  It shares no code with
 * the GPU path (no headers, helpers or tables): everything below is written from the
 * paper's equations and the readings recorded with the oracle.
 *
 * Units are SI throughout.  All arithmetic is IEEE double, single-threaded, loops in
 * array order.  Every function returns 0 on success, a positive HSO_E* code otherwise.
 */
#ifndef HS_ORACLE_H
#define HS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { HSO_OK = 0, HSO_EARG = 1, HSO_ECAP = 2, HSO_ENUM = 3, HSO_ESTATE = 5 };
enum { HSO_BC_OUTFLOW = 0, HSO_BC_SPECULAR = 1, HSO_BC_INFLOW = 2 };
enum { HSO_BODY_NONE = 0, HSO_BODY_CYLINDER = 1, HSO_BODY_SPHERE = 2 };
/* What lies across a mesh edge that has no neighbour cell. */
enum { HSO_EDGE_OUTFLOW = -1, HSO_EDGE_INFLOW = -2, HSO_EDGE_WALL = -3, HSO_EDGE_SPECULAR = -4 };

/* Gas model (Sec. 4 opening paragraph: argon, VHS, d_ref, T_ref, mu_ref, omega). */
typedef struct {
    double m, d_ref, T_ref, omega, mu_ref, Pr, gamma;
} hso_gas;

/* A drifting Maxwellian macrostate: number density, mean velocity, temperature. */
typedef struct {
    double n, u[3], T;
} hso_state;

/* A body-fitted mesh (the paper's unstructured meshes, Sec. 4.2-4.5).  In 2-D, convex
 * quadrilaterals: cell k has nodes quad[4k..4k+3] counter-clockwise; edge j runs from node j
 * to node (j+1) mod 4 and nbr[4k+j] is the cell across it.  In 3-D, convex hexahedra with
 * planar faces: nodes quad[8k..8k+7], 0-3 the bottom face counter-clockwise seen from above,
 * 4-7 above them; faces (0,3,2,1), (4,5,6,7), (0,1,5,4), (1,2,6,5), (2,3,7,6), (3,0,4,7) and
 * nbr[6k+f] across face f.  Across a boundary: an HSO_EDGE_* code: OUTFLOW removes particles
 * that cross it, INFLOW also feeds the inflow state's one-way flux through it, WALL reflects
 * diffusely at body_T, SPECULAR mirrors. */
typedef struct {
    int32_t n_nodes, n_cells;
    const double *xy;                /* 2 (2-D) or 3 (3-D) per node                    */
    const int32_t *quad;             /* 4 or 8 per cell                                */
    const int32_t *nbr;              /* 4 or 6 per cell                                */
} hso_mesh;

/* One flow case on a uniform Cartesian grid (cells x-fastest).  dim = 0 is the
 * spatially homogeneous (0-D) mode: nx cells, no transport, per-cell time steps. */
typedef struct {
    int32_t dim, nx, ny, nz;
    double lo[3], h[3];              /* unused axes: h is the unit depth/area          */
    int32_t bc[6];                   /* faces -x,+x,-y,+y,-z,+z                        */
    hso_state inflow;                /* state injected through HSO_BC_INFLOW faces     */
    double slot_lo[3], slot_hi[3];   /* inflow only where the face centre lies inside  */
    int32_t body;                    /* HSO_BODY_*; diffuse wall at body_T             */
    double body_c[3], body_r, body_T;
    int32_t n_regions;               /* initial state: first region containing a cell  */
    const double *region_box;        /* 6 per region: lo[3], hi[3]                     */
    const hso_state *region_state;
    double F_N, dt_G, T_sigma;       /* particle weight, global step, (sigma c)_max T  */
    const double *dt_over_tau;       /* dim 0 only: per-cell dt_G / tau_0              */
    uint64_t seed;
    int64_t n_steady, capacity;
    int32_t n_surf;                  /* body surface elements sampled (0: none)        */
    int32_t adapt_dt;                /* 1: Eq. 26 global step, min of Eq. 25 over cells */
    const hso_mesh *mesh;            /* NULL: the grid above; else an hso_mesh (dim 2 or 3):
                                        the cells are its quads (h[2] the depth) or
                                        hexahedra; nx, ny, nz, lo, the in-plane h, bc and
                                        the slot are unused; body only frames the surface
                                        elements (its wall is the WALL edges or faces) */
} hso_case;

typedef struct hso_sim hso_sim;

/* Per-cell record of the last step, for parity checks. */
typedef struct {
    int64_t n, ncol, nacc, nrelax, ar_attempts, ar_cap;
    uint64_t acc_hash;
    double T, tau, dt_dsmc, p_relax, a_max;
    double pre_sum[4];    /* sum c_x, c_y, c_z, sum |c|^2 before the collision step */
    double post_sum[4];   /* the same after the conservation rescale               */
} hso_trace;

/* Case-wide event counters (cumulative). */
typedef struct {
    int64_t injected, removed, wall_hits, candidates, accepted, relaxed,
            ar_attempts, ar_cap, bounce_cap, inject_cap, skipped_cells;
} hso_counters;

int  hso_create(const hso_gas *gas, const hso_case *cases, int n_cases, int trace,
                hso_sim **out);
void hso_destroy(hso_sim *s);
int  hso_init_particles(hso_sim *s);                   /* Step (1)                  */
int  hso_step(hso_sim *s, int64_t n);                  /* Steps (2)-(5), n times    */
int  hso_sample_moments(hso_sim *s, int c, int mode, double *n, double *u3, double *T,
                        double *q3, int64_t *n_samples); /* Step (6); mode 1 = now  */

/* State access: positions are absolute (x,y,z per particle), velocities 3 per particle,
 * cell is the case-local cell index, particles in array order. */
int64_t hso_num_particles(const hso_sim *s, int c);
int  hso_get_state(const hso_sim *s, int c, double *x3, double *v3, int32_t *cell,
                   int64_t *id, int64_t *next_id, int64_t *step);
int  hso_set_state(hso_sim *s, int c, int64_t np, const double *x3, const double *v3,
                   const int32_t *cell, const int64_t *id, int64_t next_id, int64_t step);
int  hso_get_cells(const hso_sim *s, int c, double *vol, double *sigc_max, double *acc13,
                   int64_t *n_samples);
int  hso_set_cells(hso_sim *s, int c, const double *sigc_max, const double *acc13,
                   int64_t n_samples);
int  hso_get_trace(const hso_sim *s, int c, hso_trace *out);
/* Body surface sampling (Step (5) on the wall; the quantities of Eq. 35-36).  Element k
 * of the n_surf elements holds the wall points whose polar angle from the upstream
 * stagnation direction -x lies in [k, k+1) pi / n_surf (a cylinder's upper and lower
 * halves together).  Raw sums per element, 7 doubles, over the sampled steps: reflections,
 * sum dP.n, sum dP.t, sum dE, sum dP (x, y, z); dP = m F_N (c_in - c_out) is the momentum
 * a reflection gives the wall, dE = m F_N (|c_in|^2 - |c_out|^2) / 2 its energy, n the
 * outward normal and t the unit tangent of growing polar angle at the hit point.
 * hso_surface_sample turns them into time averages: per element 8 doubles (mid angle,
 * area, p, tau, q, C_p, C_f, C_h) and per case 5 (force x, y, z per unit time, C_D, C_L),
 * with the inflow state as freestream (coefficients 0 when it has no speed). */
/* Global time step (Eq. 26).  With adapt_dt the step after step s uses the minimum over
 * the case's active cells (N >= 2, T > 0) of the Eq. 25 local step from step s's Step (3)
 * moments (the first step uses dt_G; a step without active cells keeps the last value);
 * otherwise dt_G throughout.  Inflow counts scale with the step.  hso_step_dt gives the
 * step the next hso_step will use and the sampled time (sum of the steps of the sampled
 * steps); hso_set_step_dt sets both (state import). */
int  hso_step_dt(const hso_sim *s, int c, double *dt_next, double *t_sampled);
int  hso_set_step_dt(hso_sim *s, int c, double dt, double t_sampled);
/* "Ratio of DSMC" per cell from the time-averaged moments (n, U, T of Step (6)):
 * Dt_DSMC / Dt_G = 1 if Dt_c <= tau, else tau / Dt_c (Eq. 27), with tau = mu(T) / (n k T)
 * (Eq. 10) and Dt_c from Eq. 25 (0-D: the cell's own step); 0 where a cell has no
 * samples. */
int  hso_dsmc_ratio(const hso_sim *s, int c, double *ratio);
int  hso_get_surface(const hso_sim *s, int c, double *sums7);
int  hso_set_surface(hso_sim *s, int c, const double *sums7);
int  hso_surface_sample(const hso_sim *s, int c, double *elem8, double *body5, int64_t *n_samples);
int  hso_get_counters(const hso_sim *s, int c, hso_counters *out);
int64_t hso_num_cells(const hso_sim *s, int c);
int64_t hso_num_faces(const hso_sim *s, int c);
int  hso_face_info(const hso_sim *s, int c, int32_t *cell, int32_t *side, double *lambda);

/* Building blocks exposed for the pin tests. */
void   hso_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void   hso_draw(uint64_t seed, uint32_t stream, uint64_t entity, uint32_t step,
                uint32_t draw, uint32_t out[4]);
double hso_uniform(uint32_t w);
uint32_t hso_index(uint32_t w, uint32_t n);
double hso_sigma_c(const hso_gas *g, double cr);
double hso_viscosity(const hso_gas *g, double T);
double hso_mean_free_path(const hso_gas *g, double n, double T);
double hso_inflow_number_flux(const hso_gas *g, const hso_state *st, const double nrm[3]);
/* flux-weighted normal speed draw (units of 1/beta), 4 words per attempt */
double hso_sample_normal_speed(double s, const uint32_t *words, int n_attempts, int *used);
/* Moments of a velocity set with the unbiased estimators of Step (3). */
int    hso_cell_moments(const hso_gas *g, int64_t N, const double *v3, double F_N,
                        double vol, double U[3], double *T, double Q[3]);
/* Shakhov AR sampling of one thermal velocity with the given draw words
 * (5 words per attempt: R1..R4, R5).  Returns attempts used (negative if capped). */
int    hso_shakhov_sample(const hso_gas *g, double T, double p, const double Q[3],
                          double a_max, const uint32_t *words, int n_attempts, double C[3]);
/* Timescale split of Step (4): returns dt_dsmc, dt_sbgk for given dt_c, tau, dt_G. */
void   hso_split(double dt_c, double tau, double dt_G, double *dt_dsmc, double *dt_sbgk);
/* Number of 16^dim sub-cell centres of a cell outside the body. */
int64_t hso_cut_count(const hso_case *c, int i, int j, int k);

#ifdef __cplusplus
}
#endif
#endif
