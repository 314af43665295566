// hs_common.hpp -- data layout shared by the host runtime and the gfx950 kernels.
//
// One sim holds a batch of cases flattened into one global cell range and one particle
// array.  Particles are structure-of-arrays in two ping-pong buffers; the step counter on
// the device selects which one is current (step & 1), so every launch of a step has
// fixed arguments and can be replayed from a graph.
#pragma once
#include <stdint.h>

#include "../../include/hs.h"

namespace hsk {

constexpr int kMaxCases = 256;
constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;   // +inf as double bits
constexpr int kSurfCopies = 16;     // copies of the wall sums, so few atomics share an address
constexpr int kMaxBounce = 8;        // body reflections per particle per step
constexpr int kMaxCross = 4096;      // mesh edge crossings per particle per step
constexpr int kMaxShakhov = 64;      // Shakhov acceptance-rejection attempts
constexpr int kMaxInjectAR = 64;     // inflow normal-speed attempts
constexpr int kMaxPosTry = 64;       // initial-position attempts in a cut cell
constexpr int kSub = 16;             // sub-cells per axis of the cut-cell volume rule
constexpr int kBlock = 256;          // threads per block of the streaming kernels

// Size classes of the block-per-cell collide kernel (cells above the tile kernel's limit):
// class 0 up to kCapBlockMid particles, 1 up to kCapBlockMax, 2 up to kCapBlockLds (the
// densest worked on in LDS), 3 above.  Each class has its own list of cells, built by the
// scan, so a launch for one class visits only its own cells.
constexpr int kCapBlockMid = 512;
constexpr int kCapBlockMax = 2048;   // powers of two: the bitonic sort pads to one
constexpr int kCapBlockLds = 4096;
constexpr int kDenseClasses = 4;
constexpr int dense_class(int n)
{
    return n <= kCapBlockMid ? 0 : n <= kCapBlockMax ? 1 : n <= kCapBlockLds ? 2 : 3;
}
// Lower bound (exclusive) of the particles of a cell of class k, given the tile limit.
constexpr int dense_class_floor(int k, int cap_wave)
{
    return k == 0 ? cap_wave : k == 1 ? kCapBlockMid : k == 2 ? kCapBlockMax : kCapBlockLds;
}

// Philox streams and per-step draw indices (shared numbering of the method's draws).
enum : uint32_t { kStreamParticle = 0, kStreamCell = 1, kStreamFace = 2, kStreamInit = 3 };
enum : uint32_t { kDrawRelax = 0, kDrawShakhov = 1, kDrawBounce = 200, kDrawInjectTime = 300 };

// Error bits of the device error word.
enum : uint32_t {
    kErrCapacity = 1u,      // particle capacity exceeded
    kErrNumeric = 4u,       // non-finite moment / velocity
    kErrState = 8u          // internal inconsistency (recomputed move disagrees)
};

struct GasDev {
    double m, R, Pr, gamma, mu_ref, T_ref, omega;
    double K_vhs, vhs_exp;  // sigma_T c_r = K c_r^(2 - 2 omega)
};

struct CaseDev {
    int32_t dim, n[3];
    int32_t cell0, ncells;          // global cell range [cell0, cell0 + ncells)
    int32_t face0, nfaces;          // global inflow-face range
    int32_t region0, nregions;
    int32_t bc[6];
    int32_t body;
    uint32_t seed_lo, seed_hi;
    int64_t n_steady, capacity;
    double lo[3], h[3], dt_over_h[3];
    double body_c[3], body_r, body_T;
    double F_N, dt_G, L_cell, sigc0, tau0;
    double in_n, in_u[3], in_T;
    int32_t bb_lo[3], bb_hi[3];     // cell-index box around the body (1-cell margin)
    int32_t surf0, n_surf;          // body surface elements: first of the batch, count
    int32_t adapt_dt;               // 1: Eq. 26 global step
    int32_t mesh;                   // 1: cells are quads of the mesh arrays of Ctx
    double inv_n[2];                // 1 / n_x and 1 / (n_x n_y): cell index -> (i, j, k)
};

struct FaceDev {
    int32_t cell;       // global boundary cell
    int32_t side;       // grid: 0..5 = -x,+x,-y,+y,-z,+z; mesh: the cell's edge 0..3
    int32_t case_id;
    int32_t local;      // face index within the case (Philox entity)
    double lambda;      // expected entering particles per step
};

struct StateDev {
    double n, u[3], T;
};

struct Globals {
    int64_t step;
    int32_t n_live;          // particles in the current buffer
    int32_t n_total;         // after injection
    int32_t n_new;           // after the sort
    int32_t spare;
    uint32_t err;
    uint32_t halt;
    int32_t n_inject;        // particles injected this step
    int32_t n_work;          // particles routed to the body-reflection kernel
    int32_t n_tiles;         // tiles of the collide kernel this step
    int32_t pad;
    int32_t case_tile0[kMaxCases + 1];   // first tile of each case (tiles never span cases)
    int64_t next_id[kMaxCases];
    int64_t inj_id_base[kMaxCases];
    int64_t n_samples[kMaxCases];
    long long counters[kMaxCases][HS_NUM_COUNTERS];
    double dt_cur[kMaxCases];                // global step of the current step
    unsigned long long dt_next[kMaxCases];   // Eq. 26 minimum so far (bits of a positive double)
    double t_sampled[kMaxCases];             // sum of the global steps of the sampled steps
    int32_t n_big[kDenseClasses];            // cells of each size class of the block-per-cell kernel
};

// Cell trace record (same field order as hs_trace).
struct TraceDev {
    int64_t n, ncol, nacc, nrelax, ar_attempts, ar_cap;
    uint64_t acc_hash;
    double T, tau, dt_dsmc, p_relax, a_max;
    double pre_sum[4];
    double post_sum[4];
};
static_assert(sizeof(TraceDev) == sizeof(hs_trace), "trace layout");

// Particle state.  A particle's id is kept as its low 32 bits: every live id of a case is one
// of the case's last 2^32 ids (below its next id), so the full id is the largest value below
// the case's next id with those bits (full_id).
struct PartBuf {
    void *pos[3];
    void *vel[3];
    int32_t *cell;
    uint32_t *id;
};

constexpr int64_t full_id(uint32_t low, int64_t next_id)
{
    return next_id - (int64_t)(uint32_t)((uint32_t)next_id - low);
}

// Everything a kernel needs, passed by value.
struct Ctx {
    const CaseDev *cases;
    const FaceDev *faces;
    const double *region_box;
    const StateDev *region_state;
    const double *dt_cell;        // per global cell (0-D cases), else unused
    GasDev gas;
    PartBuf buf[2];
    int32_t *newcell, *slot, *perm;
    int32_t *count, *cstart;      // per cell; cstart has ncells_total + 1 entries
    double *sigc, *acc, *vol;     // (sigma c)_max, 13 sums per cell, fluid volume
    double *cellrec;              // 16 doubles per cell: scalars of the collision stage
    double *surf;                 // kSurfCopies x (7 sums per body surface element, all cases)
    int32_t *face_cnt, *face_start;
    int32_t *scan_part;
    int32_t *big_list;            // the cells of size class k at big_off[k] .. big_off[k + 1]
    int32_t big_off[kDenseClasses + 1];
    int32_t *tile_cell;           // first cell of each collide tile (n_tiles + 1 entries)
    int32_t *tile_case;           // case of each tile (tiles never span cases)
    int32_t *work;                // body worklist (particle indices)
    TraceDev *trace;              // nullptr unless tracing
    // quad meshes (nullptr without a mesh case): node coordinates (2 per node, all cases),
    // per global cell its 4 global node ids, the 4 neighbours (global cell or hs_edge code)
    // and (volume, L_cell)
    const double *mxy;
    const int32_t *mquad, *mnbr;
    const double *mgeo;
    // hexahedral meshes (nullptr without one): node coordinates (3 per node), per global cell
    // its 8 global node ids and 8 neighbour words (faces 0-5, then 2 unused)
    const double *hxyz;
    const int32_t *hnode, *hnbr;
    Globals *g;
    int32_t n_cases, n_faces, ncells_total, cap_wave;   // cap_wave: densest cell of the tile kernel
    int32_t cap_block, precision, tile_w, dim_max;   // cap_block: densest cell worked on in LDS; dim_max: largest case dimension
    int32_t n_surf_total;         // surface elements of the batch (one copy)
    int64_t capacity;             // total particle capacity of the batch
    // launch shapes (blocks per grid; 0 = the built-in default), chosen by the autotuner
    int32_t grid[HS_NUM_KERNELS];
};

// Launchers (defined in hs_kernels.hip).
struct Launch {
    static void init_cells(const Ctx &c, void *stream);
    static void init_count(const Ctx &c, void *stream);
    static void init_fill(const Ctx &c, void *stream);
    static void init_finish(const Ctx &c, void *stream);
    static void scan_cells(const Ctx &c, void *stream, int build_big);
    static void tile_table(const Ctx &c, void *stream);
    static void inject(const Ctx &c, void *stream);
    static void move_count(const Ctx &c, void *stream, int any_body);
    static void scatter(const Ctx &c, void *stream);
    static void gather(const Ctx &c, void *stream);
    static void scalars(const Ctx &c, void *stream);
    static void collide(const Ctx &c, void *stream);
    static void dense(const Ctx &c, void *stream);
    static void finish_step(const Ctx &c, void *stream);
    static void philox(uint64_t seed, uint32_t stream_id, uint64_t e0, uint32_t step,
                       uint32_t draw, int64_t n, uint32_t *out, void *stream);
};

void launch_moments_now(const Ctx &c, void *stream, int case_id, int ncells, double *out8);
void launch_build_big(const Ctx &c, void *stream);
void launch_finalize(const Ctx &c, void *stream, int case_id, int ncells, double *out8);
void launch_surface_finalize(const Ctx &c, void *stream, int case_id, double *out);
void launch_dsmc_ratio(const Ctx &c, void *stream, int case_id, int ncells, double *out);
void launch_surface_reduce(const Ctx &c, void *stream, int case_id, double *out);
// The library's fixed scratch array on the current device (HS_STATIC_SCRATCH_BYTES): its
// device address and size; 0 on success, else the HIP error code.
int static_scratch(void **ptr, size_t *bytes);
int cap_wave();
int tile_width();
int cap_block(int precision);

}  // namespace hsk
