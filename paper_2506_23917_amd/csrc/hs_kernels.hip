// hs_kernels.hip -- gfx950 kernels of one step of the hybrid SP-Shakhov / DSMC particle
// update (arXiv 2506.23917, Sec. 3.2 Steps 1-5) and their launchers.
//
// Step pipeline (all on one stream, fixed launch arguments):
//   inject_count / inject_scan / inject_fill   inflow faces -> new particles appended
//   move_count     per particle: free flight + walls -> new cell, atomic per-cell slot
//   scan_*         exclusive scan of the cell counts -> cell_start, dense-cell list
//   scatter        perm[cell_start[c] + slot] = source index
//   collide_wave   one wavefront per cell (<= cap_wave particles): gather the cell's
//                  sources, restore their array order, re-run their move, write the new
//                  sorted state; moments, split, NTC chain, Shakhov, rescale, sampling
//   collide_block  the same with a 256-thread block for each dense cell
//   finish_step    live count, step counter, sample counters
#include "hs_device.hpp"

#include <mutex>
#include <type_traits>

namespace hsk {

// ------------------------------------------------------------------------------------
// team helpers (TEAM = 64: one wavefront; TEAM = 256: one block)
// ------------------------------------------------------------------------------------

template <int TEAM>
__device__ __forceinline__ void team_sync()
{
    if constexpr (TEAM == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Sum K doubles over the team; every thread ends with the same bits (butterfly adds are
// commutative pairwise, the cross-wave step uses one fixed order).
template <int TEAM, int K>
__device__ __forceinline__ void team_sum(double (&v)[K], double *red)
{
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] = v[k] + __shfl_xor(v[k], off, 64);
    }
    if constexpr (TEAM > 64) {
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) red[w * K + k] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = red[k];
            for (int ww = 1; ww < TEAM / 64; ++ww) s = s + red[ww * K + k];
            v[k] = s;
        }
    }
}

template <int TEAM, int K>
__device__ __forceinline__ void team_sum_i(long long (&v)[K], long long *red)
{
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    if constexpr (TEAM > 64) {
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) red[w * K + k] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            long long s = 0;
            for (int ww = 0; ww < TEAM / 64; ++ww) s += red[ww * K + k];
            v[k] = s;
        }
    }
}

template <int TEAM>
__device__ __forceinline__ bool team_any(bool p, int *redi)
{
    const bool w = __any(p);
    if constexpr (TEAM == 64) {
        return w;
    } else {
        __syncthreads();
        if (threadIdx.x == 0) redi[0] = 0;
        __syncthreads();
        if (w && (threadIdx.x & 63) == 0) atomicOr(&redi[0], 1);
        __syncthreads();
        return redi[0] != 0;
    }
}

// Add `val` to base[key] for every active lane, one atomic per distinct key in the wave.
__device__ __forceinline__ void wave_add(long long *base, int stride, int key, int idx, long long val, bool active)
{
    unsigned long long pending = __ballot(active && val != 0);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int k0 = __shfl(key, leader, 64);
        const bool mine = ((pending >> (threadIdx.x & 63)) & 1ull) && key == k0;
        long long s = mine ? val : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if ((threadIdx.x & 63) == leader) atomicAdd((unsigned long long *)&base[(long long)k0 * stride + idx], (unsigned long long)s);
        pending &= ~__ballot(mine);
    }
}

__device__ __forceinline__ void raise_error(Globals *g, uint32_t bits)
{
    atomicOr(&g->err, bits);
    atomicExch(&g->halt, 1u);
}

// Load base[byte_off / sizeof(T)] with a 32-bit byte offset (uniform base in SGPRs, the
// offset in one VGPR).
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, uint32_t byte_off)
{
    return *(const T *)((const char *)base + byte_off);
}

template <typename P>
struct Parts {
    P *pos[3];
    P *vel[3];
    int32_t *cell;
    uint32_t *id;             // low 32 bits of the ids (full_id)
    __device__ explicit Parts(const PartBuf &b)
    {
        for (int a = 0; a < 3; ++a) {
            pos[a] = (P *)b.pos[a];
            vel[a] = (P *)b.vel[a];
        }
        cell = b.cell;
        id = b.id;
    }
};

// ------------------------------------------------------------------------------------
// Step (1): initialisation
// ------------------------------------------------------------------------------------

__device__ inline const StateDev *region_of(const Ctx &C, const CaseDev &cs, const int ijk[3])
{
    if (cs.nregions <= 0) return nullptr;
    if (cs.dim == 0) return &C.region_state[cs.region0];
    for (int r = 0; r < cs.nregions; ++r) {
        const double *b = &C.region_box[6 * (cs.region0 + r)];
        bool in = true;
        for (int a = 0; a < 3; ++a) if (a < cs.dim) {
            const double ctr = cs.lo[a] + ((double)ijk[a] + 0.5) * cs.h[a];
            if (!(ctr >= b[a] && ctr < b[3 + a])) in = false;
        }
        if (in) return &C.region_state[cs.region0 + r];
    }
    return nullptr;
}

// Region of a hexahedron: the first box holding the mean of its eight nodes.
__device__ inline const StateDev *region_of_hex(const Ctx &C, const CaseDev &cs, int g)
{
    if (cs.nregions <= 0) return nullptr;
    double P[8][3];
    hex_nodes(C, g, P);
    double mc[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 8; ++j)
        for (int a = 0; a < 3; ++a) mc[a] = mc[a] + P[j][a];
    for (int a = 0; a < 3; ++a) mc[a] = 0.125 * mc[a];
    for (int r = 0; r < cs.nregions; ++r) {
        const double *b = &C.region_box[6 * (cs.region0 + r)];
        if (mc[0] >= b[0] && mc[0] < b[3] && mc[1] >= b[1] && mc[1] < b[4] && mc[2] >= b[2] && mc[2] < b[5])
            return &C.region_state[cs.region0 + r];
    }
    return nullptr;
}

// Region of a mesh cell: the first box holding the mean of its four nodes.
__device__ inline const StateDev *region_of_mesh(const Ctx &C, const CaseDev &cs, int g)
{
    if (cs.nregions <= 0) return nullptr;
    if (cs.dim == 3) return region_of_hex(C, cs, g);
    double P[4][2];
    mesh_nodes(C, g, P);
    double mc[2] = {0.0, 0.0};
    for (int j = 0; j < 4; ++j) {
        mc[0] = mc[0] + P[j][0];
        mc[1] = mc[1] + P[j][1];
    }
    mc[0] = 0.25 * mc[0];
    mc[1] = 0.25 * mc[1];
    for (int r = 0; r < cs.nregions; ++r) {
        const double *b = &C.region_box[6 * (cs.region0 + r)];
        if (mc[0] >= b[0] && mc[0] < b[3] && mc[1] >= b[1] && mc[1] < b[4]) return &C.region_state[cs.region0 + r];
    }
    return nullptr;
}

__global__ void k_init_cells(Ctx C, int fill)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= C.ncells_total) return;
    const CaseDev &cs = C.cases[case_of(C, g)];
    const int lc = g - cs.cell0;
    int ijk[3];
    cell_ijk(cs, lc, ijk);
    int full = 1;
    for (int a = 0; a < 3; ++a) if (a < cs.dim) full *= kSub;
    const double vfull = cs.h[0] * cs.h[1] * cs.h[2];
    double vol = vfull;
    if (cs.mesh) vol = C.mgeo[2 * (size_t)g];
    else if (cs.body != HS_BODY_NONE && cs.dim > 0) vol = (double)cut_count(cs, ijk) / (double)full * vfull;
    C.vol[g] = vol;
    C.sigc[g] = cs.sigc0;
    for (int j = 0; j < 13; ++j) C.acc[13 * (size_t)g + j] = 0.0;
    int N = 0;
    if (fill && vol > 0.0) {
        const StateDev *st = cs.mesh ? region_of_mesh(C, cs, g) : region_of(C, cs, ijk);
        if (st && st->n > 0.0) {
            const W4 w = draw(cs, kStreamInit, (uint64_t)lc, 0, 0);
            N = (int)floor(st->n * vol / cs.F_N + unid(w.x));
        }
    }
    C.count[g] = N;
}

template <typename P>
__global__ __launch_bounds__(64) void k_init_fill(Ctx C)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= C.ncells_total) return;
    const int s = C.cstart[g], N = C.cstart[g + 1] - s;
    if (N == 0) return;
    if ((long long)s + N > C.capacity) {
        raise_error(C.g, kErrCapacity);
        return;
    }
    const CaseDev &cs = C.cases[case_of(C, g)];
    const int lc = g - cs.cell0;
    int ijk[3];
    cell_ijk(cs, lc, ijk);
    const StateDev *st = cs.mesh ? region_of_mesh(C, cs, g) : region_of(C, cs, ijk);
    Parts<P> B(C.buf[0]);
    const int64_t id0 = (int64_t)s - C.cstart[cs.cell0];
    const double a = sqrt(2.0 * C.gas.R * st->T);
    double Pq[4][2], jmax = 0.0;
    if (cs.mesh && cs.dim == 2) {
        mesh_nodes(C, g, Pq);
        for (int cu = 0; cu < 2; ++cu)
            for (int cw = 0; cw < 2; ++cw) {
                double X[2];
                const double jc = bilinear(Pq, (double)cu, (double)cw, X);
                if (jc > jmax) jmax = jc;
            }
    }
    for (int q = 0; q < N; ++q) {
        double xr[3] = {0.0, 0.0, 0.0};
        if (cs.mesh && cs.dim == 3) {
            // uniform in the hexahedron: uniform in its bounding box, kept when inside every face
            double Ph[8][3], lo[3], hi[3], xc[3] = {0.0, 0.0, 0.0}, X[3];
            hex_nodes(C, g, Ph);
            for (int j = 0; j < 8; ++j)
                for (int a = 0; a < 3; ++a) {
                    if (j == 0 || Ph[j][a] < lo[a]) lo[a] = Ph[j][a];
                    if (j == 0 || Ph[j][a] > hi[a]) hi[a] = Ph[j][a];
                    xc[a] = xc[a] + Ph[j][a];
                }
            bool placed = false;
            for (int t = 0; t < kMaxPosTry && !placed; ++t) {
                const W4 w = draw(cs, kStreamInit, (uint64_t)lc, 0, (uint32_t)(1 + 128 * q + t));
                const uint32_t ww[3] = {w.x, w.y, w.z};
                for (int a = 0; a < 3; ++a) X[a] = lo[a] + unid(ww[a]) * (hi[a] - lo[a]);
                placed = true;
                for (int f = 0; f < 6 && placed; ++f) {
                    const double *A;
                    double nf[3];
                    hex_face(Ph, f, A, nf);
                    const double d[3] = {A[0] - X[0], A[1] - X[1], A[2] - X[2]};
                    if (dot3(d, nf) < 0.0) placed = false;
                }
            }
            if (!placed)
                for (int a = 0; a < 3; ++a) X[a] = 0.125 * xc[a];
            for (int a = 0; a < 3; ++a) xr[a] = X[a] - Ph[0][a];
        } else if (cs.mesh) {
            // uniform in the quad: the bilinear map accepted with probability J / J_max
            double X[2];
            bool placed = false;
            for (int t = 0; t < kMaxPosTry && !placed; ++t) {
                const W4 w = draw(cs, kStreamInit, (uint64_t)lc, 0, (uint32_t)(1 + 128 * q + t));
                const double J = bilinear(Pq, unid(w.x), unid(w.y), X);
                placed = unid(w.z) * jmax < J;
            }
            if (!placed) bilinear(Pq, 0.5, 0.5, X);
            xr[0] = X[0] - Pq[0][0];
            xr[1] = X[1] - Pq[0][1];
        } else if (cs.dim > 0) {
            bool placed = false;
            for (int t = 0; t < kMaxPosTry && !placed; ++t) {
                const W4 w = draw(cs, kStreamInit, (uint64_t)lc, 0, (uint32_t)(1 + 128 * q + t));
                const uint32_t ww[3] = {w.x, w.y, w.z};
                double X[3] = {0.0, 0.0, 0.0};
                for (int d = 0; d < 3; ++d) if (d < cs.dim) {
                    xr[d] = unid(ww[d]);
                    X[d] = cs.lo[d] + ((double)ijk[d] + xr[d]) * cs.h[d];
                }
                placed = !in_body(cs, X);
            }
            if (!placed) {
                const int s2n = cs.dim >= 3 ? kSub : 1, s1n = cs.dim >= 2 ? kSub : 1;
                for (int s2 = 0; s2 < s2n && !placed; ++s2)
                    for (int s1 = 0; s1 < s1n && !placed; ++s1)
                        for (int s0 = 0; s0 < kSub && !placed; ++s0) {
                            const int sub[3] = {s0, s1, s2};
                            double X[3] = {0.0, 0.0, 0.0};
                            for (int d = 0; d < 3; ++d) if (d < cs.dim) {
                                xr[d] = ((double)sub[d] + 0.5) / kSub;
                                X[d] = cs.lo[d] + ((double)ijk[d] + xr[d]) * cs.h[d];
                            }
                            placed = !in_body(cs, X);
                        }
            }
        }
        const W4 w = draw(cs, kStreamInit, (uint64_t)lc, 0, (uint32_t)(1 + 128 * q + 64));
        double s1, c1, s3, c3;
        sincospi(2.0 * unid(w.x), &s1, &c1);
        sincospi(2.0 * unid(w.z), &s3, &c3);
        const double r2 = sqrt(-log(unid(w.y))), r4 = sqrt(-log(unid(w.w)));
        const double C3[3] = {a * c1 * r2, a * c3 * r4, a * s3 * r4};
        const size_t i = (size_t)s + q;
        for (int d = 0; d < 3; ++d) {
            P x = (P)xr[d];
            if (!cs.mesh && !(x < (P)1)) x = Real<P>::below_one();
            if (d < cs.dim) B.pos[d][i] = x;
            B.vel[d][i] = (P)(st->u[d] + C3[d]);
        }
        B.cell[i] = g;
        B.id[i] = (uint32_t)(id0 + q);
    }
}

__global__ void k_init_finish(Ctx C, int64_t step0)
{
    Globals *G = C.g;
    const int t = threadIdx.x;
    for (int c = t; c < C.n_cases; c += blockDim.x) {
        const CaseDev &cs = C.cases[c];
        const int64_t np = (int64_t)C.cstart[cs.cell0 + cs.ncells] - C.cstart[cs.cell0];
        G->next_id[c] = np;
        G->n_samples[c] = 0;
        G->dt_cur[c] = cs.dt_G;
        G->dt_next[c] = kInfBits;
        G->t_sampled[c] = 0.0;
        for (int k = 0; k < HS_NUM_COUNTERS; ++k) G->counters[c][k] = 0;
        if (np > cs.capacity) raise_error(G, kErrCapacity);
    }
    if (t == 0) {
        G->step = step0;
        G->n_live = C.cstart[C.ncells_total];
        G->n_total = G->n_live;
        G->n_new = G->n_live;
        for (int k = 0; k < kDenseClasses; ++k) G->n_big[k] = 0;
        G->n_inject = 0;
        if (G->n_live > C.capacity) raise_error(G, kErrCapacity);
    }
}

// Append the lanes' dense cells g (n particles, above the tile limit; `dense` false for the
// other lanes) to the lists of their size classes: one atomic per class and wave, called by
// every lane of the wave alike.  A class-k list holds at most capacity / (floor_k + 1) cells,
// its reserved length.
__device__ __forceinline__ void add_dense(const Ctx &C, int g, int n, bool dense)
{
    if (!__any(dense)) return;
    const int cls = dense ? dense_class(n) : -1;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < kDenseClasses; ++k) {
        const unsigned long long m = __ballot(cls == k);
        if (!m) continue;
        const int leader = __ffsll((long long)m) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&C.g->n_big[k], __popcll(m));
        base = __shfl(base, leader, 64);
        if (cls == k) {
            const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
            if (C.big_off[k] + slot < C.big_off[k + 1]) C.big_list[C.big_off[k] + slot] = g;
            else raise_error(C.g, kErrState);
        }
    }
}

// ------------------------------------------------------------------------------------
// Exclusive scan of per-cell counts (three phases: block sums, scan of block sums,
// block-local scan + offset).  Each block covers kScanTile cells.
// ------------------------------------------------------------------------------------

constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int block_excl_scan(int v, int *lds, int &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    __syncthreads();
    if (lane == 63) lds[w] = incl;
    __syncthreads();
    int before = 0;
    const int nw = blockDim.x >> 6;
    total = 0;
    for (int k = 0; k < nw; ++k) {
        if (k < w) before += lds[k];
        total += lds[k];
    }
    return before + incl - v;
}

__global__ void k_scan_reduce(Ctx C)
{
    if (C.g->halt) return;
    __shared__ int lds[16];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int g = base + k;
        if (g < C.ncells_total) s += C.count[g];
    }
    int total;
    block_excl_scan(s, lds, total);
    if (threadIdx.x == 0) C.scan_part[blockIdx.x] = total;
}

__global__ void k_scan_parts(Ctx C, int nparts)
{
    if (C.g->halt) return;
    __shared__ int lds[16];
    int carry = 0;
    for (int base = 0; base < nparts; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const int v = i < nparts ? C.scan_part[i] : 0;
        int total;
        const int ex = block_excl_scan(v, lds, total);
        __syncthreads();
        if (i < nparts) C.scan_part[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) C.scan_part[nparts] = carry;
}

// Collide tiles never span two cases, so a case is tiled exactly as it would be alone (its
// cell sums then run in the same order in any batch).  Tile t of case k covers the cells c
// of the case whose local weight w(c) = (cstart[c] - cstart[cell0]) + 4 (c - cell0), which
// strictly increases, lies in [t TW, (t+1) TW); tile_cell[] holds the first cell of every
// tile of the batch and, after the last, ncells.
__global__ void k_case_tiles(Ctx C)
{
    if (C.g->halt) return;
    __shared__ int lds[16];
    Globals *G = C.g;
    const long long tw = C.tile_w;
    int carry = 0;
    for (int base = 0; base < C.n_cases; base += blockDim.x) {
        const int k = base + threadIdx.x;
        int v = 0;
        if (k < C.n_cases) {
            const CaseDev &cs = C.cases[k];
            const long long W = (long long)(C.cstart[cs.cell0 + cs.ncells] - C.cstart[cs.cell0]) + 4ll * cs.ncells;
            v = (int)((W + tw - 1) / tw);
        }
        int total;
        const int ex = block_excl_scan(v, lds, total);
        __syncthreads();
        if (k < C.n_cases) G->case_tile0[k] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        G->case_tile0[C.n_cases] = carry;
        G->n_tiles = carry;
        C.tile_cell[carry] = C.ncells_total;
    }
}

__global__ void k_tile_table(Ctx C)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= C.ncells_total || C.g->halt) return;
    const int k = case_of(C, g);
    const CaseDev &cs = C.cases[k];
    const long long tw = C.tile_w;
    const long long c0 = C.cstart[cs.cell0];
    const long long w0 = (C.cstart[g] - c0) + 4ll * (g - cs.cell0);
    const long long w1 = (C.cstart[g + 1] - c0) + 4ll * (g + 1 - cs.cell0);
    const int t0 = C.g->case_tile0[k], ntk = C.g->case_tile0[k + 1] - t0;
    int32_t *tc = C.tile_cell + t0;
    int32_t *tk = C.tile_case + t0;
    for (long long t = w0 / tw + 1; t <= w1 / tw; ++t) {
        tc[t] = g + 1;
        if (t < ntk) tk[t] = k;
    }
    if (g == cs.cell0) {
        tc[0] = g;
        tk[0] = k;
    }
    if (g == cs.cell0 + cs.ncells - 1 && w1 % tw != 0) tc[w1 / tw + 1] = g + 1;
}

__global__ void k_scan_final(Ctx C, int build_big, int nparts)
{
    if (C.g->halt) return;
    __shared__ int lds[16];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int g = base + k;
        v[k] = g < C.ncells_total ? C.count[g] : 0;
        s += v[k];
    }
    int total;
    int run = C.scan_part[blockIdx.x] + block_excl_scan(s, lds, total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int g = base + k;
        if (g < C.ncells_total) {
            C.cstart[g] = run;
            C.count[g] = 0;
        }
        if (build_big) add_dense(C, g, v[k], g < C.ncells_total && v[k] > C.cap_wave);
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int all = C.scan_part[nparts];
        C.cstart[C.ncells_total] = all;
        C.g->n_new = all;
    }
}

// ------------------------------------------------------------------------------------
// Inflow injection (Step 2 freestream boundaries)
// ------------------------------------------------------------------------------------

__global__ void k_inject_count(Ctx C)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= C.n_faces || C.g->halt) return;
    const FaceDev fd = C.faces[f];
    const CaseDev &cs = C.cases[fd.case_id];
    const W4 w = draw(cs, kStreamFace, (uint64_t)fd.local, (uint32_t)C.g->step, 0);
    // lambda is per dt_G; an adapted global step (Eq. 26) scales it
    const double lam = cs.adapt_dt ? fd.lambda * (C.g->dt_cur[fd.case_id] / cs.dt_G) : fd.lambda;
    C.face_cnt[f] = (int)floor(lam + unid(w.x));
}

__global__ void k_inject_scan(Ctx C)
{
    if (C.g->halt) return;
    __shared__ int lds[16];
    Globals *G = C.g;
    int carry = 0;
    for (int base = 0; base < C.n_faces; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const int v = i < C.n_faces ? C.face_cnt[i] : 0;
        int total;
        const int ex = block_excl_scan(v, lds, total);
        __syncthreads();
        if (i < C.n_faces) C.face_start[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) C.face_start[C.n_faces] = carry;
    __syncthreads();
    for (int c = threadIdx.x; c < C.n_cases; c += blockDim.x) {
        const CaseDev &cs = C.cases[c];
        const int inj = C.face_start[cs.face0 + cs.nfaces] - C.face_start[cs.face0];
        const int64_t live = (int64_t)C.cstart[cs.cell0 + cs.ncells] - C.cstart[cs.cell0];
        if (live + inj > cs.capacity) raise_error(G, kErrCapacity);
        G->inj_id_base[c] = G->next_id[c];
        G->next_id[c] += inj;
        G->counters[c][HS_CNT_INJECTED] += inj;
    }
    if (threadIdx.x == 0) {
        G->n_inject = carry;
        G->n_total = G->n_live + carry;
        if ((int64_t)G->n_total > C.capacity) raise_error(G, kErrCapacity);
    }
}

// One wavefront per inflow face; lanes stride over the face's new particles.  The launch
// bound lets the hexahedral placement keep its nodes in registers (without it the compiler
// assumes 1024-thread blocks, caps the kernel at 128 VGPRs and spills about 700).
template <typename P>
__global__ __launch_bounds__(kBlock) void k_inject_fill(Ctx C)
{
    const int f = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (f >= C.n_faces || C.g->halt) return;
    const int cnt = C.face_cnt[f];
    if (cnt == 0) return;
    const FaceDev fd = C.faces[f];
    const CaseDev &cs = C.cases[fd.case_id];
    const uint32_t st = (uint32_t)C.g->step;
    Parts<P> S(C.buf[C.g->step & 1]);
    const int a = fd.side / 2;
    const double sg = (fd.side % 2 == 0) ? 1.0 : -1.0;
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    const double beta = 1.0 / sqrt(2.0 * C.gas.R * cs.in_T);
    const double ath = sqrt(2.0 * C.gas.R * cs.in_T);
    const double sn = sg * cs.in_u[a] * beta;
    const int64_t slot0 = (int64_t)C.g->n_live + C.face_start[f];
    const int64_t id0 = C.g->inj_id_base[fd.case_id] + (C.face_start[f] - C.face_start[cs.face0]);
    long long capped = 0;
    if (cs.mesh && cs.dim == 3) {
        // a hexahedron's face: inward normal n = -nf / |nf|; tangents t1, t2 by Gram-Schmidt
        // from the two axes other than the one n is most aligned with; points from the face's
        // bilinear map (origin: the corner of smallest t1 + t2 coordinate, u towards its
        // neighbour of larger t1 coordinate) accepted with probability J / J_max
        double Ph[8][3], Pf[4][3];
        hex_nodes(C, fd.cell, Ph);
        for (int j = 0; j < 4; ++j)
            for (int a = 0; a < 3; ++a) Pf[j][a] = Ph[kHexFace[fd.side][j]][a];
        const double *A;
        double nfv[3];
        hex_face(Ph, fd.side, A, nfv);
        const double ln = sqrt(dot3(nfv, nfv));
        const double n[3] = {-nfv[0] / ln, -nfv[1] / ln, -nfv[2] / ln};
        int ax = 0;
        for (int a = 1; a < 3; ++a) if (fabs(n[a]) > fabs(n[ax])) ax = a;
        const int a1 = ax == 0 ? 1 : 0, a2 = ax == 2 ? 1 : 2;
        double t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
        t1[a1] = 1.0;
        t2[a2] = 1.0;
        const double p1 = n[a1];
        for (int a = 0; a < 3; ++a) t1[a] = t1[a] - p1 * n[a];
        const double l1 = sqrt(dot3(t1, t1));
        for (int a = 0; a < 3; ++a) t1[a] = t1[a] / l1;
        const double q2 = n[a2], r2 = t1[a2];
        for (int a = 0; a < 3; ++a) t2[a] = t2[a] - q2 * n[a] - r2 * t1[a];
        const double l2 = sqrt(dot3(t2, t2));
        for (int a = 0; a < 3; ++a) t2[a] = t2[a] / l2;
        int o = 0;
        for (int j = 1; j < 4; ++j)
            if (dot3(t1, Pf[j]) + dot3(t2, Pf[j]) < dot3(t1, Pf[o]) + dot3(t2, Pf[o])) o = j;
        int ju = (o + 1) & 3, jv = (o + 3) & 3;
        if (dot3(t1, Pf[jv]) > dot3(t1, Pf[ju])) { const int tmp = ju; ju = jv; jv = tmp; }
        const double *Po = Pf[o], *Pu = Pf[ju], *Pv = Pf[jv], *Pw = Pf[(o + 2) & 3];
        auto jac = [&](double uu, double vq) {
            double du[3], dv[3];
            for (int a = 0; a < 3; ++a) {
                du[a] = (1.0 - vq) * (Pu[a] - Po[a]) + vq * (Pw[a] - Pv[a]);
                dv[a] = (1.0 - uu) * (Pv[a] - Po[a]) + uu * (Pw[a] - Pu[a]);
            }
            const double cr[3] = {du[1] * dv[2] - du[2] * dv[1], du[2] * dv[0] - du[0] * dv[2],
                                  du[0] * dv[1] - du[1] * dv[0]};
            return sqrt(dot3(cr, cr));
        };
        double jmax = 0.0;
        for (int cu = 0; cu < 2; ++cu)
            for (int cv = 0; cv < 2; ++cv) {
                const double jc = jac((double)cu, (double)cv);
                if (jc > jmax) jmax = jc;
            }
        const double snm = dot3(cs.in_u, n) * beta;
        const double ut1 = dot3(cs.in_u, t1), ut2 = dot3(cs.in_u, t2);
        for (int q = lane; q < cnt; q += 64) {
            const uint32_t base = (uint32_t)(1 + 128 * q);
            double u = 0.5, vv = 0.5;
            for (int r = 0; r < 32; ++r) {
                const W4 wp = draw(cs, kStreamFace, (uint64_t)fd.local, st, r == 0 ? base : base + 66 + (uint32_t)r);
                const double uu = unid(wp.x), vq = unid(wp.y);
                if (unid(wp.z) * jmax < jac(uu, vq)) { u = uu; vv = vq; break; }
            }
            double X[3];
            for (int a = 0; a < 3; ++a)
                X[a] = (1.0 - u) * (1.0 - vv) * Po[a] + u * (1.0 - vv) * Pu[a] + u * vv * Pw[a] + (1.0 - u) * vv * Pv[a];
            const W4 wv = draw(cs, kStreamFace, (uint64_t)fd.local, st, base + 1);
            const double rr = sqrt(-log(unid(wv.y)));
            double sn2, cs2;
            sincospi(2.0 * unid(wv.x), &sn2, &cs2);
            const double v1 = ut1 + ath * cs2 * rr, v2 = ut2 + ath * sn2 * rr;
            int used;
            const double z = normal_speed(cs, (uint32_t)fd.local, st, base + 2, snm, used);
            if (used < 0) ++capped;
            const size_t i = (size_t)(slot0 + q);
            for (int a = 0; a < 3; ++a) {
                S.pos[a][i] = (P)(X[a] - Ph[0][a]);
                S.vel[a][i] = (P)(n[a] * z / beta + t1[a] * v1 + t2[a] * v2);
            }
            S.cell[i] = fd.cell;
            S.id[i] = (uint32_t)(id0 + q);
        }
    } else if (cs.mesh) {
        // a mesh edge: inward normal n = (-e_y, e_x) / |e|, in-plane tangent t = (-n_y, n_x)
        // or its opposite (t_x + t_y >= 0), points along +t from the end of smaller t.x
        double Pq[4][2];
        mesh_nodes(C, fd.cell, Pq);
        const double *A = Pq[fd.side], *Bn = Pq[(fd.side + 1) & 3];
        const double ex = Bn[0] - A[0], ey = Bn[1] - A[1];
        const double len = sqrt(ex * ex + ey * ey);
        const double nx = -ey / len, ny = ex / len;
        double tx = -ny, ty = nx;
        if (tx + ty < 0.0) { tx = -tx; ty = -ty; }
        const double *S0 = A, *E0 = Bn;
        if (Bn[0] * tx + Bn[1] * ty < A[0] * tx + A[1] * ty) { S0 = Bn; E0 = A; }
        const double snm = (cs.in_u[0] * nx + cs.in_u[1] * ny) * beta;
        const double ut = cs.in_u[0] * tx + cs.in_u[1] * ty;
        for (int q = lane; q < cnt; q += 64) {
            const uint32_t base = (uint32_t)(1 + 128 * q);
            const W4 wp = draw(cs, kStreamFace, (uint64_t)fd.local, st, base);
            const double frac = unid(wp.x);
            const double X0 = S0[0] + frac * (E0[0] - S0[0]), X1 = S0[1] + frac * (E0[1] - S0[1]);
            const W4 wv = draw(cs, kStreamFace, (uint64_t)fd.local, st, base + 1);
            const double rr = sqrt(-log(unid(wv.y)));
            double sn2, cs2;
            sincospi(2.0 * unid(wv.x), &sn2, &cs2);
            const double vt = ut + ath * cs2 * rr;
            const double vz = cs.in_u[2] + ath * sn2 * rr;
            int used;
            const double z = normal_speed(cs, (uint32_t)fd.local, st, base + 2, snm, used);
            if (used < 0) ++capped;
            const size_t i = (size_t)(slot0 + q);
            S.pos[0][i] = (P)(X0 - Pq[0][0]);
            S.pos[1][i] = (P)(X1 - Pq[0][1]);
            S.vel[0][i] = (P)(nx * z / beta + tx * vt);
            S.vel[1][i] = (P)(ny * z / beta + ty * vt);
            S.vel[2][i] = (P)vz;
            S.cell[i] = fd.cell;
            S.id[i] = (uint32_t)(id0 + q);
        }
    } else
    for (int q = lane; q < cnt; q += 64) {
        const uint32_t base = (uint32_t)(1 + 128 * q);
        double xr[3] = {0.0, 0.0, 0.0}, v[3];
        const W4 wp = draw(cs, kStreamFace, (uint64_t)fd.local, st, base);
        for (int t = 0; t < cs.dim; ++t)
            if (t != a) xr[t] = unid(t == t1 ? wp.x : wp.y);
        xr[a] = (fd.side % 2 == 0) ? 0.0 : 1.0;
        const W4 wv = draw(cs, kStreamFace, (uint64_t)fd.local, st, base + 1);
        const double rr = sqrt(-log(unid(wv.y)));
        double sn2, cs2;
        sincospi(2.0 * unid(wv.x), &sn2, &cs2);
        v[t1] = cs.in_u[t1] + ath * cs2 * rr;
        v[t2] = cs.in_u[t2] + ath * sn2 * rr;
        int used;
        const double z = normal_speed(cs, (uint32_t)fd.local, st, base + 2, sn, used);
        if (used < 0) ++capped;
        v[a] = sg * z / beta;
        const size_t i = (size_t)(slot0 + q);
        for (int d = 0; d < 3; ++d) {
            P x = (P)xr[d];
            if (d != a && !(x < (P)1)) x = Real<P>::below_one();
            if (d < cs.dim) S.pos[d][i] = x;
            S.vel[d][i] = (P)v[d];
        }
        S.cell[i] = fd.cell;
        S.id[i] = (uint32_t)(id0 + q);
    }
    if (capped) atomicAdd((unsigned long long *)&C.g->counters[fd.case_id][HS_CNT_INJECT_CAP], (unsigned long long)capped);
}

// Counter sums of one wave by case.  Lane l holds counter base + (l & 7) of slot l >> 3
// (eight cases at a time).  Lanes count privately; when the wave moves to a tile of another
// case their counts are summed over the wave into that case's slot, and the flush adds each
// slot with one atomic per lane, so no address takes an atomic per lane or per tile.
struct CaseTally {
    long long val;
    int slot_case;
    int nslot;                          // uniform over the wave
};

template <int K>
__device__ __forceinline__ void tally_flush(const Ctx &C, CaseTally &T, int base)
{
    const int k = threadIdx.x & 7;
    if (T.slot_case >= 0 && k < K && T.val != 0)
        atomicAdd((unsigned long long *)&C.g->counters[T.slot_case][base + k], (unsigned long long)T.val);
    T.val = 0;
    T.slot_case = -1;
    T.nslot = 0;
}

// Adds the wave's sums of v[] to case cid (every lane of the wave calls it).
template <int K>
__device__ __forceinline__ void tally_add(const Ctx &C, CaseTally &T, int cid, int base, const long long (&v)[K])
{
    static_assert(K <= 8, "eight counters per slot");
    long long tot[K];
    bool any = false;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        long long x = v[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        tot[j] = x;
        any = any || x != 0;
    }
    if (!any || cid < 0) return;
    const int lane = threadIdx.x & 63;
    const unsigned long long hit = __ballot(T.slot_case == cid);
    int slot;
    if (hit) {
        slot = (__ffsll((long long)hit) - 1) >> 3;
    } else {
        if (T.nslot == 8) tally_flush<K>(C, T, base);
        slot = T.nslot++;
        if ((lane >> 3) == slot) T.slot_case = cid;
    }
    if ((lane >> 3) == slot) {
        const int k = lane & 7;
        long long a = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j == k) a = tot[j];
        T.val += a;
    }
}

// ------------------------------------------------------------------------------------
// Free transport and cell counts (Step 2 -> Step 3 histogram)
// ------------------------------------------------------------------------------------

// Wave-aggregated slot allocation: one atomic per distinct destination cell in the wave;
// returns this lane's slot in its cell (order within a cell is arbitrary; the collide
// kernels restore the stable order).  The lanes are grouped by cell first (one uniform pass
// per distinct cell, each lane keeping its group's lane mask); a lane's rank is the number
// of its group's lanes below it, and the group's lowest lane takes the group's slots.
__device__ __forceinline__ int wave_slot(int32_t *count, int nc, bool want)
{
    unsigned long long pending = __ballot(want);
    unsigned long long mine = 0ull;
    while (pending) {
        const int l0 = __ffsll((long long)pending) - 1;
        const int c0 = __builtin_amdgcn_readlane(nc, l0);
        const bool in = want && nc == c0;
        const unsigned long long same = __ballot(in);
        if (in) mine = same;
        pending &= ~same;
    }
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned int)(mine >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((unsigned int)mine, 0u));
    int old = 0;
    if (want && rank == 0) old = atomicAdd(&count[nc], __popcll(mine));
    old = __shfl(old, __ffsll((long long)mine) - 1, 64);
    return old + rank;
}

// Straight flight of particle i of case cs (state already loaded): the moved position
// written back in place (velocity too when a wall changed it), the new cell returned in nc
// (-1: left the domain); to_body when the path may meet the body.
template <typename P>
__device__ __forceinline__ void move_fast_one(const CaseDev &cs, const Parts<P> &S, int i, int g, P (&xr)[3],
                                              P (&v)[3], uint32_t st, int n_live, double dt, const int64_t *next_id,
                                              int &nc, bool &to_body)
{
    if (cs.dim == 0) {
        nc = g;
        return;
    }
    const bool full = i < n_live;
    double t = dt;
    if (!full) t = dt * unid(draw(cs, kStreamParticle, (uint64_t)full_id(S.id[i], *next_id), st, kDrawInjectTime).x);
    bool vchg = false;
    const int nl = flight<P>(cs, g - cs.cell0, xr, v, t, full, vchg);
    if (nl == -2) {
        to_body = true;
    } else if (nl >= 0) {
        nc = cs.cell0 + nl;
        for (int a = 0; a < 3; ++a) if (a < cs.dim) S.pos[a][i] = xr[a];
        if (vchg)
            for (int a = 0; a < 3; ++a) if (a < cs.dim) S.vel[a][i] = v[a];
    }
}

// Every particle of the grid cases: straight flight with specular / open walls, new cell and
// slot recorded.  Particles whose path may meet the body go to a worklist for k_move_body;
// waves of mesh cases are left to k_move_mesh.  Cases are contiguous in the particle array
// (the sorted live part, then the injected particles case by case), so a wave nearly always
// lies in one case: that case's fields are then uniform (scalar loads) and its removals are
// counted per lane and summed once per case change; a wave spanning two cases takes the
// general path.
template <typename P>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_move_fast(Ctx C)
{
    Globals *G = C.g;
    if (G->halt) return;
    const int n_total = G->n_total, n_live = G->n_live;
    const uint32_t st = (uint32_t)G->step;
    const Parts<P> S(C.buf[G->step & 1]);
    const int stride = gridDim.x * blockDim.x;
    CaseTally tally{0, -1, 0};
    long long removed[1] = {0};          // this lane's removals in case rcase (uniform waves)
    int rcase = -1;
    for (int base = blockIdx.x * blockDim.x; base < n_total; base += stride) {
        const int i = base + threadIdx.x;
        const bool valid = i < n_total;       // the valid lanes of a wave are a prefix
        int g = 0;
        P xr[3] = {(P)0, (P)0, (P)0}, v[3] = {(P)0, (P)0, (P)0};
        if (valid) {
            // state loads first (guarded by the batch's largest dimension, not the case's)
            g = S.cell[i];
#pragma unroll
            for (int a = 0; a < 3; ++a) if (a < C.dim_max) xr[a] = S.pos[a][i];
#pragma unroll
            for (int a = 0; a < 3; ++a) v[a] = S.vel[a][i];
        }
        const int cu = case_of(C, __builtin_amdgcn_readfirstlane(g));
        const CaseDev &csu = case_const(C, cu);
        const bool one = __all(!valid || (g >= csu.cell0 && g < csu.cell0 + csu.ncells));
        int nc = -1;
        bool to_body = false, mine = false;
        if (one) {
            if (csu.mesh) continue;           // a mesh case's wave: k_move_mesh moves it
            mine = valid;
            if (valid) move_fast_one<P>(csu, S, i, g, xr, v, st, n_live, const_read(&G->dt_cur[cu]), &G->next_id[cu], nc, to_body);
            if (cu != rcase) {
                tally_add<1>(C, tally, rcase, HS_CNT_REMOVED, removed);
                removed[0] = 0;
                rcase = cu;
            }
            removed[0] += (valid && !to_body && nc < 0) ? 1 : 0;
        } else {
            int cid = cu;
            if (valid) {
                cid = case_of(C, g);
                mine = C.cases[cid].mesh == 0;
                if (mine) move_fast_one<P>(C.cases[cid], S, i, g, xr, v, st, n_live, G->dt_cur[cid], &G->next_id[cid], nc, to_body);
            }
            wave_add(&G->counters[0][0], HS_NUM_COUNTERS, cid, HS_CNT_REMOVED, 1, mine && !to_body && nc < 0);
        }
        // worklist of body candidates
        {
            const int lane = threadIdx.x & 63;
            const unsigned long long m = __ballot(to_body);
            if (m) {
                int basew = 0;
                const int leader = __ffsll((long long)m) - 1;
                if (lane == leader) basew = atomicAdd(&G->n_work, __popcll(m));
                basew = __shfl(basew, leader, 64);
                if (to_body) C.work[basew + __popcll(m & ((1ull << lane) - 1ull))] = i;
            }
        }
        const bool counted = mine && !to_body && nc >= 0;
        if (mine && !to_body) C.newcell[i] = nc;
        const int myslot = wave_slot(C.count, nc, counted);
        if (counted) C.slot[i] = myslot;
    }
    tally_add<1>(C, tally, rcase, HS_CNT_REMOVED, removed);
    tally_flush<1>(C, tally, HS_CNT_REMOVED);
}

// Every particle of the mesh cases: face-to-face tracking (move_mesh through quads, move_hex
// through hexahedra), new cell and slot.  Waves of grid cases pass straight through
// (k_move_fast moves them).
template <typename P>
__global__ __launch_bounds__(kBlock) void k_move_mesh(Ctx C)
{
    Globals *G = C.g;
    if (G->halt) return;
    const int n_total = G->n_total, n_live = G->n_live;
    const uint32_t st = (uint32_t)G->step;
    const Parts<P> S(C.buf[G->step & 1]);
    const int stride = gridDim.x * blockDim.x;
    const int copy = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kSurfCopies);
    for (int base = blockIdx.x * blockDim.x; base < n_total; base += stride) {
        const int i = base + threadIdx.x;
        const bool valid = i < n_total;
        const int g = valid ? S.cell[i] : 0;
        const int cu = case_of(C, __builtin_amdgcn_readfirstlane(g));
        const CaseDev &csu = case_const(C, cu);
        const bool one = __all(!valid || (g >= csu.cell0 && g < csu.cell0 + csu.ncells));
        if (one && !csu.mesh) continue;
        const int cid = one ? cu : (valid ? case_of(C, g) : cu);
        const CaseDev &cs = C.cases[cid];
        const bool mine = valid && cs.mesh;
        int nc = -1;
        MoveStats ms{0, 0};
        if (mine) {
            P xr[3] = {S.pos[0][i], S.pos[1][i], (P)0}, v[3] = {S.vel[0][i], S.vel[1][i], S.vel[2][i]};
            const bool full = i < n_live;
            int64_t id = -1;
            const double dt = G->dt_cur[cid];
            double t = dt;
            const IdSrc ids{&S.id[i], G->next_id[cid]};
            if (!full) {
                id = ids.get();
                t = dt * unid(draw(cs, kStreamParticle, (uint64_t)id, st, kDrawInjectTime).x);
            }
            double *surf = (cs.n_surf > 0 && G->step >= cs.n_steady)
                               ? C.surf + 7 * (size_t)copy * (size_t)C.n_surf_total : nullptr;
            if (cs.dim == 3) {
                xr[2] = S.pos[2][i];
                nc = move_hex<P>(C, cs, g, xr, v, id, ids, t, st, ms, surf);
            } else {
                nc = move_mesh<P>(C, cs, g, xr, v, id, ids, t, st, ms, surf);
            }
            if (nc >= 0) {
                S.pos[0][i] = xr[0];
                S.pos[1][i] = xr[1];
                if (cs.dim == 3) S.pos[2][i] = xr[2];
                for (int a = 0; a < 3; ++a) S.vel[a][i] = v[a];
            }
            C.newcell[i] = nc;
        }
        const int myslot = wave_slot(C.count, nc, mine && nc >= 0);
        if (mine && nc >= 0) C.slot[i] = myslot;
        wave_add(&G->counters[0][0], HS_NUM_COUNTERS, cid, HS_CNT_REMOVED, 1, mine && nc < 0);
        wave_add(&G->counters[0][0], HS_NUM_COUNTERS, cid, HS_CNT_WALL_HITS, ms.hits, mine);
        wave_add(&G->counters[0][0], HS_NUM_COUNTERS, cid, HS_CNT_BOUNCE_CAP, ms.capped, mine);
    }
}

// Worklist particles: the full move with FP64 body reflections (diffuse wall).
template <typename P>
__global__ __launch_bounds__(kBlock) void k_move_body(Ctx C)
{
    Globals *G = C.g;
    if (G->halt) return;
    const int nw = G->n_work, n_live = G->n_live;
    const uint32_t st = (uint32_t)G->step;
    const Parts<P> S(C.buf[G->step & 1]);
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < nw; base += stride) {
        const int w = base + threadIdx.x;
        const bool valid = w < nw;
        int nc = -1, cid = 0, i = 0;
        MoveStats ms{0, 0};
        if (valid) {
            i = C.work[w];
            const int g = S.cell[i];
            cid = case_of(C, g);
            const CaseDev &cs = C.cases[cid];
            P xr[3], v[3];
            for (int a = 0; a < 3; ++a) if (a < cs.dim) xr[a] = S.pos[a][i];
            for (int a = 0; a < 3; ++a) v[a] = S.vel[a][i];
            const bool full = i < n_live;
            int64_t id = -1;
            const double dt = G->dt_cur[cid];
            double t = dt;
            const IdSrc ids{&S.id[i], G->next_id[cid]};
            if (!full) {
                id = ids.get();
                t = dt * unid(draw(cs, kStreamParticle, (uint64_t)id, st, kDrawInjectTime).x);
            }
            // wall sums of the body (Step (5) on the surface) in sampled steps
            // (each wave adds to one of kSurfCopies copies of the sums)
            const int copy = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kSurfCopies);
            double *surf = (cs.n_surf > 0 && G->step >= cs.n_steady)
                               ? C.surf + 7 * (size_t)copy * (size_t)C.n_surf_total : nullptr;
            const int nl = move_particle<P>(C.gas, cs, g - cs.cell0, xr, v, id, ids, t, full, st, ms, surf);
            if (nl >= 0) {
                nc = cs.cell0 + nl;
                for (int a = 0; a < 3; ++a) if (a < cs.dim) S.pos[a][i] = xr[a];
                for (int a = 0; a < 3; ++a) S.vel[a][i] = v[a];
            }
            C.newcell[i] = nc;
        }
        const int myslot = wave_slot(C.count, nc, valid && nc >= 0);
        if (valid && nc >= 0) C.slot[i] = myslot;
        wave_add(&G->counters[0][0], HS_NUM_COUNTERS, cid, HS_CNT_REMOVED, 1, valid && nc < 0);
        wave_add(&G->counters[0][0], HS_NUM_COUNTERS, cid, HS_CNT_WALL_HITS, ms.hits, valid);
        wave_add(&G->counters[0][0], HS_NUM_COUNTERS, cid, HS_CNT_BOUNCE_CAP, ms.capped, valid);
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter(Ctx C)
{
    Globals *G = C.g;
    if (G->halt) return;
    const int n_total = G->n_total;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += gridDim.x * blockDim.x) {
        const int nc = C.newcell[i];
        if (nc >= 0) C.perm[C.cstart[nc] + C.slot[i]] = i;
    }
}

// ------------------------------------------------------------------------------------
// Collision stage (Step 3 moments, Step 4, Step 5)
// ------------------------------------------------------------------------------------

struct CellCounts {
    long long cand, acc, relax, ar, arcap, skipped;
};

// Shakhov acceptance-rejection draw (Eq. 17-18) for one relaxing particle.
template <typename P>
__device__ __forceinline__ int shakhov_draw(uint32_t sd0, uint32_t sd1, int64_t id, uint32_t st, const P *par,
                                            P one_m_pr, P Cv[3])
{
    const P ath = par[5], p = par[3], RT = par[4], am = par[6];
#pragma unroll 1
    for (int a = 0; a < kMaxShakhov; ++a) {
        const W4 w = draw_s(sd0, sd1, kStreamParticle, (uint64_t)id, st, kDrawShakhov + 2 * a);
        const W4 w5 = draw_s(sd0, sd1, kStreamParticle, (uint64_t)id, st, kDrawShakhov + 2 * a + 1);
        P s1, c1, s3, c3;
        Real<P>::sc2pi(Real<P>::uni(w.x), &s1, &c1);
        Real<P>::sc2pi(Real<P>::uni(w.z), &s3, &c3);
        const P r2 = Real<P>::sq(-Real<P>::ln(Real<P>::uni(w.y)));
        const P r4 = Real<P>::sq(-Real<P>::ln(Real<P>::uni(w.w)));
        Cv[0] = ath * c1 * r2;
        Cv[1] = ath * c3 * r4;
        Cv[2] = ath * s3 * r4;
        const P c2 = Cv[0] * Cv[0] + Cv[1] * Cv[1] + Cv[2] * Cv[2];
        const P qc = par[0] * Cv[0] + par[1] * Cv[1] + par[2] * Cv[2];
        const P A = (P)1 + one_m_pr * qc / ((P)5 * p * RT) * (c2 / RT - (P)5);
        if (A / am > Real<P>::uni(w5.x)) return a + 1;
    }
    return -kMaxShakhov;
}

__device__ __forceinline__ void flush_counts(const Ctx &C, int cid, CellCounts &cc)
{
    long long *cnt = &C.g->counters[cid][0];
    if (cc.cand) atomicAdd((unsigned long long *)&cnt[HS_CNT_CANDIDATES], (unsigned long long)cc.cand);
    if (cc.acc) atomicAdd((unsigned long long *)&cnt[HS_CNT_ACCEPTED], (unsigned long long)cc.acc);
    if (cc.relax) atomicAdd((unsigned long long *)&cnt[HS_CNT_RELAXED], (unsigned long long)cc.relax);
    if (cc.ar) atomicAdd((unsigned long long *)&cnt[HS_CNT_AR_ATTEMPTS], (unsigned long long)cc.ar);
    if (cc.arcap) atomicAdd((unsigned long long *)&cnt[HS_CNT_AR_CAP], (unsigned long long)cc.arcap);
    if (cc.skipped) atomicAdd((unsigned long long *)&cnt[HS_CNT_SKIPPED_CELLS], (unsigned long long)cc.skipped);
    cc = CellCounts{0, 0, 0, 0, 0, 0};
}

// Kernel-end flush of every lane's counts: one atomic per counter and distinct case in the
// wave (same-address atomics from every lane of every block would serialise in L2).
__device__ __forceinline__ void wave_flush_counts(const Ctx &C, int cid, CellCounts &cc)
{
    long long *base = &C.g->counters[0][0];
    const bool on = cid >= 0;
    wave_add(base, HS_NUM_COUNTERS, cid, HS_CNT_CANDIDATES, cc.cand, on);
    wave_add(base, HS_NUM_COUNTERS, cid, HS_CNT_ACCEPTED, cc.acc, on);
    wave_add(base, HS_NUM_COUNTERS, cid, HS_CNT_RELAXED, cc.relax, on);
    wave_add(base, HS_NUM_COUNTERS, cid, HS_CNT_AR_ATTEMPTS, cc.ar, on);
    wave_add(base, HS_NUM_COUNTERS, cid, HS_CNT_AR_CAP, cc.arcap, on);
    wave_add(base, HS_NUM_COUNTERS, cid, HS_CNT_SKIPPED_CELLS, cc.skipped, on);
    cc = CellCounts{0, 0, 0, 0, 0, 0};
}

// ---- wavefront-tile collide kernel ----------------------------------------------------

// Inclusive prefix sum over the wavefront.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
    }
    return v;
}

// One round of segmented sums: lane holds K values of slot base + lane; `head` is the first
// lane of that slot's cell within the round (cells are contiguous runs of slots).  After
// the segmented scan, the owner lane of each cell pulls its run's sum from `tail` (the last
// lane of its run in this round, or -1) and adds it to acc.  The order of additions is
// fixed, so results are reproducible.
template <int K>
__device__ __forceinline__ void seg_round(double (&x)[K], int head, int tail, double (&acc)[K])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const bool take = lane - off >= head;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double y = __shfl_up(x[k], off, 64);
            if (take) x[k] = x[k] + y;
        }
    }
    const int src = tail >= 0 ? tail : lane;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double y = __shfl(x[k], src, 64);
        if (tail >= 0) acc[k] = acc[k] + y;
    }
}

// XCD-aware order of the tiles.  Workgroups are dealt to the chip's 8 XCDs in turn (block b
// runs on XCD b mod 8), and each XCD has its own L2.  Neighbouring tiles read the same source
// cache lines (a cell's particles come from the cells around it, which belong to tiles a row
// apart), so each XCD takes whole chunks of kTileChunk consecutive tiles, chunk c going to
// XCD c mod 8, and its blocks sweep them in order.  The grid is a multiple of 8.
constexpr int kXcds = 8;
constexpr int kTileChunk = 256;
// FP32-mixed tiles of the tile collision kernel with more cells than this send their Step (5)
// sums in address order (see the kernel); fewer, wider groups send their own.  FP64 tiles always
// send their own: that kernel runs two waves per SIMD and is bound by instruction issue, its
// per-lane adds overlap with its arithmetic, and the address-order walk measured slower there.
constexpr int kSampSpread = 16;

// Eq. 26: fold a wave's smallest local step of case cid (lanes hold their own minima, +inf
// where none) into the case's minimum for the next global step; one atomic per wave.
__device__ __forceinline__ void wave_flush_dtmin(const Ctx &C, int cid, double dtmin)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dtmin = fmin(dtmin, __shfl_xor(dtmin, off, 64));
    if ((threadIdx.x & 63) == 0 && cid >= 0 && dtmin < INFINITY)
        atomicMin(&C.g->dt_next[cid], (unsigned long long)__double_as_longlong(dtmin));
}

// Tile of the p-th position in this block's XCD sequence (increasing in p).
__device__ __forceinline__ int xcd_tile(int p, int xcd)
{
    const int chunk = p / kTileChunk;
    return (chunk * kXcds + xcd) * kTileChunk + (p - chunk * kTileChunk);
}

// Table entries of a tile: first cell, end cell, case.  The tile kernels load those of the
// next tile while they work on the current one (uniform loads, through the scalar cache).
struct TileRef {
    int cb, ce, ci;
};

__device__ __forceinline__ TileRef tile_ref(const Ctx &C, int t, int ntiles)
{
    TileRef r{0, 0, 0};
    if (t < ntiles) {
        r.cb = const_read(C.tile_cell + t);
        r.ce = const_read(C.tile_cell + t + 1);
        r.ci = const_read(C.tile_case + t);
    }
    return r;
}

// Per-cell record written by k_cell_scalars for the tile kernel (16 doubles per cell):
// U[3], T, P_relax, (sigma c)_max, N_col, active, Shakhov parameters Q[3], p, RT,
// sqrt(2RT), A_max.
enum : int {
    kRecU = 0, kRecT = 3, kRecPr = 4, kRecScm = 5, kRecNcol = 6, kRecAct = 7, kRecPar = 8, kRecLen = 16
};

// Tiles of the collision stage: a 64-thread block takes the cells whose weight
// w(c) = cell_start[c] + 4 c falls in [t TW, (t+1) TW): at most TW/4 = 64 cells and TW + D
// particles; cells denser than D go to k_collide_dense.  This kernel restores the stable
// order of each cell's particles (source order) and writes the sorted state.  Its time is
// load latency: in FP32 it runs at eight waves per SIMD (64 VGPRs, a few spilled), in FP64
// at four (eight would spill 32 VGPRs).
template <typename P, int TW, int D>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(P) == 4 ? 8 : 4, 8))) void k_sort_gather(Ctx C)
{
    constexpr int MAXC = TW / 4;
    constexpr int MAXP = TW + D;
    __shared__ __attribute__((aligned(16))) int32_t s_src[MAXP];   // source of each scatter slot
    __shared__ int32_t s_dsrc[MAXP];      // source of each destination slot
    __shared__ uint8_t s_lc[MAXP];
    __shared__ int32_t c_start[MAXC], c_off[MAXC + 1];
    // first slot of every non-empty cell as a bit, and the cell of each non-empty ordinal:
    // the cell of slot s is s_ord[(non-empty cells starting at or before s) - 1]
    constexpr int RW = (MAXP + 63) / 64;
    __shared__ unsigned long long s_first[RW];
    __shared__ uint8_t s_ord[MAXC];
    Globals *G = C.g;
    if (G->halt) return;
    const int lane = threadIdx.x;
    const int64_t step = G->step;
    const uint32_t st = (uint32_t)step;
    const Parts<P> S(C.buf[step & 1]);
    const Parts<P> Dd(C.buf[(step & 1) ^ 1]);
    const bool use_perm = C.perm != nullptr;
    const int ntiles = G->n_tiles;
    const int NC = C.ncells_total;

    const int xcd = blockIdx.x % kXcds, nbx = gridDim.x / kXcds;
    int pos = blockIdx.x / kXcds;
    int t = xcd_tile(pos, xcd);
    TileRef nx = tile_ref(C, t, ntiles);
    while (t < ntiles) {
        const TileRef cur = nx;
        pos += nbx;
        t = xcd_tile(pos, xcd);
        nx = tile_ref(C, t, ntiles);
        const int cb = cur.cb;
        const int ncl = cur.ce - cb;
        if (ncl < 0 || ncl > MAXC || cb < 0 || cb + ncl > NC || cur.ci < 0 || cur.ci >= C.n_cases) {
            if (lane == 0) raise_error(G, kErrState);
            return;
        }
        const int dim = case_const(C, cur.ci).dim;
        // owner lane = local cell
        const bool own = lane < ncl;
        int n = 0, start = 0;
        bool dense = false;
        const int g = cb + lane;
        if (own) {
            start = C.cstart[g];
            n = C.cstart[g + 1] - start;
            dense = n > D;
            c_start[lane] = start;
        }
        const int nn = (own && !dense) ? n : 0;
        const int incl = wave_incl_scan(nn);
        const int off = incl - nn;
        const int np = __shfl(incl, 63, 64);
        if (own) c_off[lane] = off;
        if (lane == 0) c_off[ncl] = np;
        if (lane < RW) s_first[lane] = 0ull;
        team_sync<64>();
        const bool ne = nn > 0;
        const unsigned long long mne = __ballot(ne);
        if (ne) {
            atomicOr(&s_first[off >> 6], 1ull << (off & 63));
            s_ord[__popcll(mne & ((1ull << lane) - 1ull))] = (uint8_t)lane;
        }
        team_sync<64>();
        // slots -> cells, sources (all index loads issued before any is used)
        constexpr int R = RW;
        {
            int pidx[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int s = lane + 64 * r;
                pidx[r] = -1;
                // non-empty cells starting before this row (their starts increase with the lane)
                const int before = __popcll(__ballot(ne && off < 64 * r));
                if (s < np) {
                    const unsigned long long wbits = s_first[r];
                    const int a = s_ord[before + __popcll(wbits & ((2ull << lane) - 1ull)) - 1];
                    s_lc[s] = (uint8_t)a;
                    pidx[r] = c_start[a] + (s - c_off[a]);
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (pidx[r] >= 0) pidx[r] = use_perm ? C.perm[pidx[r]] : pidx[r];
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (pidx[r] >= 0) s_src[lane + 64 * r] = pidx[r];
        }
        team_sync<64>();
        // stable order inside each cell: a source's rank among its cell's sources is its
        // place (sources are distinct); the slots then hold sources in destination order.
        // The cell's sources are read four at a time (aligned 16-byte LDS reads) and all
        // counted; the few words of the first and last row outside the cell are counted again
        // and taken off (words past np are read, added and subtracted alike).
        static_assert(MAXP % 4 == 0, "whole 16-byte rows");
        for (int s = lane; s < np; s += 64) {
            const int lc = s_lc[s];
            const int o = c_off[lc], e = c_off[lc + 1];
            const int src = s_src[s];
            const int u0 = o >> 2, u1 = (e + 3) >> 2;
            int rk = 0;
            const int4 *q = reinterpret_cast<const int4 *>(s_src);
            for (int u = u0; u < u1; ++u) {
                const int4 w = q[u];
                rk += (int)(w.x < src) + (int)(w.y < src) + (int)(w.z < src) + (int)(w.w < src);
            }
            for (int k = u0 << 2; k < o; ++k) rk -= (int)(s_src[k] < src);
            for (int k = e; k < (u1 << 2); ++k) rk -= (int)(s_src[k] < src);
            s_dsrc[o + rk] = src;
        }
        team_sync<64>();
        // gather by destination slot (neighbouring lanes write neighbouring particles and,
        // sources being in increasing order, mostly read neighbouring ones); the loads of a
        // group of rows are in flight together
        constexpr int RG = 4;
#pragma unroll
        for (int r0 = 0; r0 < R; r0 += RG) {
            P gv[RG][3], gp[RG][3];
            uint32_t gid[RG];
#pragma unroll
            for (int q = 0; q < RG; ++q) {
                const int d = lane + 64 * (r0 + q);
                if (r0 + q < R && d < np) {
                    const uint32_t src = (uint32_t)s_dsrc[d];
#pragma unroll
                    for (int c = 0; c < 3; ++c) gv[q][c] = ld_off(S.vel[c], src * (uint32_t)sizeof(P));
                    gid[q] = ld_off(S.id, src * 4u);
#pragma unroll
                    for (int a2 = 0; a2 < 3; ++a2)
                        gp[q][a2] = a2 < dim ? ld_off(S.pos[a2], src * (uint32_t)sizeof(P)) : (P)0;
                }
            }
#pragma unroll
            for (int q = 0; q < RG; ++q) {
                const int d = lane + 64 * (r0 + q);
                if (r0 + q < R && d < np) {
                    const int lc = s_lc[d];
                    const size_t dst = (size_t)c_start[lc] + (d - c_off[lc]);
#pragma unroll
                    for (int a2 = 0; a2 < 3; ++a2)
                        if (a2 < dim) Dd.pos[a2][dst] = gp[q][a2];
                    Dd.cell[dst] = cb + lc;
                    Dd.id[dst] = gid[q];
                    Dd.vel[0][dst] = gv[q][0];
                    Dd.vel[1][dst] = gv[q][1];
                    Dd.vel[2][dst] = gv[q][2];
                }
            }
        }
        team_sync<64>();

    }
}

// Value held by the partner lane under a DPP lane pattern (every lane active).
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_partner_i(int x)
{
    return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
}
// DPP lane patterns: the other lane of a pair, the other pair of a quad (quad_perm), the other
// quad of an 8-lane half row (half-row mirror), the other half of a 16-lane row (row mirror).
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// Butterfly sum over each aligned group of 2^kb lanes (kb uniform in the wave).  Every lane
// of a group ends with the same bits: at each level the two partners add the same two values
// (partial sums of complementary halves).  Levels within a 16-lane row move data with DPP,
// the two wider ones with cross-lane shuffles.
template <int K>
__device__ __forceinline__ void group_sum(double (&x)[K], int kb)
{
    if (kb >= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = x[k] + dpp_partner<kDppXor1>(x[k]);
    }
    if (kb >= 2) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = x[k] + dpp_partner<kDppXor2>(x[k]);
    }
    if (kb >= 3) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = x[k] + dpp_partner<kDppHalfMirror>(x[k]);
    }
    if (kb >= 4) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = x[k] + dpp_partner<kDppMirror>(x[k]);
    }
    for (int m = 16; m < (1 << kb); m <<= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = x[k] + __shfl_xor(x[k], m, 64);
    }
}

__device__ __forceinline__ int group_sum_i(int x, int kb)
{
    if (kb >= 1) x += dpp_partner_i<kDppXor1>(x);
    if (kb >= 2) x += dpp_partner_i<kDppXor2>(x);
    if (kb >= 3) x += dpp_partner_i<kDppHalfMirror>(x);
    if (kb >= 4) x += dpp_partner_i<kDppMirror>(x);
    for (int m = 16; m < (1 << kb); m <<= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// The same with a group size per lane (groups of several sizes in one wave, each aligned to
// its size): every level up to the wave's largest group runs, and a lane adds its partner's
// value only at the levels inside its own group.
template <int K>
__device__ __forceinline__ void group_sum_v(double (&x)[K], int kb, int kbmax)
{
    if (kbmax >= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) { const double y = dpp_partner<kDppXor1>(x[k]); if (kb >= 1) x[k] = x[k] + y; }
    }
    if (kbmax >= 2) {
#pragma unroll
        for (int k = 0; k < K; ++k) { const double y = dpp_partner<kDppXor2>(x[k]); if (kb >= 2) x[k] = x[k] + y; }
    }
    if (kbmax >= 3) {
#pragma unroll
        for (int k = 0; k < K; ++k) { const double y = dpp_partner<kDppHalfMirror>(x[k]); if (kb >= 3) x[k] = x[k] + y; }
    }
    if (kbmax >= 4) {
#pragma unroll
        for (int k = 0; k < K; ++k) { const double y = dpp_partner<kDppMirror>(x[k]); if (kb >= 4) x[k] = x[k] + y; }
    }
    for (int l = 4; l < kbmax; ++l) {
#pragma unroll
        for (int k = 0; k < K; ++k) { const double y = __shfl_xor(x[k], 1 << l, 64); if (kb > l) x[k] = x[k] + y; }
    }
}

__device__ __forceinline__ int group_sum_iv(int x, int kb, int kbmax)
{
    if (kbmax >= 1) { const int y = dpp_partner_i<kDppXor1>(x); if (kb >= 1) x += y; }
    if (kbmax >= 2) { const int y = dpp_partner_i<kDppXor2>(x); if (kb >= 2) x += y; }
    if (kbmax >= 3) { const int y = dpp_partner_i<kDppHalfMirror>(x); if (kb >= 3) x += y; }
    if (kbmax >= 4) { const int y = dpp_partner_i<kDppMirror>(x); if (kb >= 4) x += y; }
    for (int l = 4; l < kbmax; ++l) { const int y = __shfl_xor(x, 1 << l, 64); if (kb > l) x += y; }
    return x;
}

// Steps (3)-(4a) of the tiles' cells: Eq. 31 moments of the sorted velocities, Eq. 10 / 25-28
// timescales and split, the NTC candidate count and the Shakhov parameters; one record per
// cell.  Each cell is served by an aligned group of 2^kb lanes (2^kb ncl <= 64): a lane sums
// every 2^kb-th particle of its cell straight from memory and the group combines the
// partial sums by a butterfly, so every lane of the group holds the cell's totals and
// derives the scalars itself; lane `sub == 0` records them.
template <typename P, int TW, int D>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_cell_scalars(Ctx C)
{
    constexpr int MAXC = TW / 4;
    Globals *G = C.g;
    if (G->halt) return;
    const int lane = threadIdx.x;
    const int64_t step = G->step;
    const uint32_t st = (uint32_t)step;
    const Parts<P> Dd(C.buf[(step & 1) ^ 1]);
    const int ntiles = G->n_tiles;
    const int NC = C.ncells_total;
    const GasDev &gas = C.gas;
    const bool tracing = C.trace != nullptr;
    long long skipped[1] = {0};
    CaseTally tally{0, -1, 0};
    int my_case = -1;
    double dtmin = INFINITY;          // smallest Eq. 25 local step of my_case's cells so far

    const int xcd = blockIdx.x % kXcds, nbx = gridDim.x / kXcds;
    int pos = blockIdx.x / kXcds;
    int t = xcd_tile(pos, xcd);
    TileRef nx = tile_ref(C, t, ntiles);
    while (t < ntiles) {
        const TileRef cur = nx;
        pos += nbx;
        t = xcd_tile(pos, xcd);
        nx = tile_ref(C, t, ntiles);
        const int cb = cur.cb;
        const int ncl = cur.ce - cb;
        const int cid = cur.ci;
        if (ncl < 0 || ncl > MAXC || cb < 0 || cb + ncl > NC || cid < 0 || cid >= C.n_cases) {
            if (lane == 0) raise_error(G, kErrState);
            return;
        }
        if (ncl == 0) continue;
        if (cid != my_case) {
            tally_add<1>(C, tally, my_case, HS_CNT_SKIPPED_CELLS, skipped);
            skipped[0] = 0;
            wave_flush_dtmin(C, my_case, dtmin);
            dtmin = INFINITY;
            my_case = cid;
        }
        const CaseDev &cs = case_const(C, cid);
        const int kb = ncl == 1 ? 6 : 6 - (32 - __clz(ncl - 1));
        const int kk = 1 << kb;
        const int gc = lane >> kb, sub = lane & (kk - 1);
        const bool own = gc < ncl;
        const int g = cb + gc;
        int start = 0, n = 0;
        double vol = 0.0, scm = 0.0;
        if (own) {
            start = C.cstart[g];
            n = C.cstart[g + 1] - start;
            vol = C.vol[g];
            scm = C.sigc[g];
        }
        const bool work = own && n <= D;
        const int nn = work ? n : 0;
        // nothing to do in a tile without particles of its own (unless trace records are kept)
        if (!tracing && !__any(nn > 0)) continue;
        const bool lead = work && sub == 0;
        const P *vx = Dd.vel[0] + start, *vy = Dd.vel[1] + start, *vz = Dd.vel[2] + start;

        // A lane's particles are i = sub, sub + kk, ...; they are read kU at a time with all
        // loads in flight before the first is used, and summed in that order.
        constexpr int kU = 2;
        auto load_u = [&](int i0, P (&bx)[kU], P (&by)[kU], P (&bz)[kU]) {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * kk;
                bx[u] = by[u] = bz[u] = (P)0;
                if (i < nn) {
                    bx[u] = vx[i];
                    by[u] = vy[i];
                    bz[u] = vz[i];
                }
            }
        };
        // Eq. 31: sums of c and |c|^2
        double s1[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i0 = sub; i0 < nn; i0 += kU * kk) {
#pragma clang fp contract(fast)
            P bx[kU], by[kU], bz[kU];
            load_u(i0, bx, by, bz);
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (i0 + u * kk < nn) {
                    const double x = (double)bx[u], y = (double)by[u], z = (double)bz[u];
                    s1[0] = s1[0] + x;
                    s1[1] = s1[1] + y;
                    s1[2] = s1[2] + z;
                    s1[3] = s1[3] + (x * x + y * y + z * z);
                }
            }
        }
        group_sum<4>(s1, kb);
        double U[3] = {0.0, 0.0, 0.0};
        if (nn > 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) U[a] = s1[a] / (double)nn;
        }
        // sums of the peculiar |C|^2 and |C|^2 C: always in FP64 (T is their first); in
        // FP32-mixed (T from the raw sums) only where the heat flux is needed
        double s2[4] = {0.0, 0.0, 0.0, 0.0};
        auto peculiar = [&](bool on) {
            if (on) {
                if constexpr (sizeof(P) == 4) {
                    // FP32 peculiar velocity and products (C = (c - U_f) - (U - U_f))
                    float uf[3], ud[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        uf[a] = (float)U[a];
                        ud[a] = (float)(U[a] - (double)uf[a]);
                    }
                    for (int i0 = sub; i0 < nn; i0 += kU * kk) {
#pragma clang fp contract(fast)
                        P bx[kU], by[kU], bz[kU];
                        load_u(i0, bx, by, bz);
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            if (i0 + u * kk < nn) {
                                const float cx = (bx[u] - uf[0]) - ud[0];
                                const float cy = (by[u] - uf[1]) - ud[1];
                                const float cz = (bz[u] - uf[2]) - ud[2];
                                const float c2 = cx * cx + cy * cy + cz * cz;
                                s2[0] = s2[0] + (double)c2;
                                s2[1] = s2[1] + (double)(c2 * cx);
                                s2[2] = s2[2] + (double)(c2 * cy);
                                s2[3] = s2[3] + (double)(c2 * cz);
                            }
                        }
                    }
                } else {
                    for (int i0 = sub; i0 < nn; i0 += kU * kk) {
#pragma clang fp contract(fast)
                        P bx[kU], by[kU], bz[kU];
                        load_u(i0, bx, by, bz);
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            if (i0 + u * kk < nn) {
                                const double cx = bx[u] - U[0], cy = by[u] - U[1], cz = bz[u] - U[2];
                                const double c2 = cx * cx + cy * cy + cz * cz;
                                s2[0] = s2[0] + c2;
                                s2[1] = s2[1] + c2 * cx;
                                s2[2] = s2[2] + c2 * cy;
                                s2[3] = s2[3] + c2 * cz;
                            }
                        }
                    }
                }
            }
            group_sum<4>(s2, kb);
        };
        if constexpr (sizeof(P) == 8) peculiar(nn >= 2);

        TraceDev *tr = (lead && tracing) ? &C.trace[g] : nullptr;
        double T = 0.0, pr = 0.0, p = 0.0, tau = 0.0, dtD = 0.0;
        bool active = false;
        if (work && nn >= 2) {
            if constexpr (sizeof(P) == 4)
                T = gas.m * (s1[3] - (s1[0] * s1[0] + s1[1] * s1[1] + s1[2] * s1[2]) / (double)nn) /
                    (3.0 * kKB * (double)(nn - 1));
            else
                T = gas.m * s2[0] / (3.0 * kKB * (double)(nn - 1));
            if (!isfinite(T)) raise_error(G, kErrNumeric);
            active = T > 0.0 && vol > 0.0;
            if (!active && lead) ++skipped[0];
        }
        if (active) {
            const double nd = (double)nn * cs.F_N / vol;
            p = nd * kKB * T;
            tau = gas.mu_ref * pow(T / gas.T_ref, gas.omega) / p;
            const double dtG = cs.dim == 0 ? C.dt_cell[g] : const_read(&G->dt_cur[cid]);
            double dtc;
            if (cs.dim == 0) {
                dtc = dtG;
            } else {
                const double um = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
                dtc = (cs.mesh ? C.mgeo[2 * (size_t)g + 1] : cs.L_cell) / (um + sqrt(gas.gamma * gas.R * T));
                if (cs.adapt_dt) dtmin = fmin(dtmin, dtc);
            }
            double dtS;
            if (dtc <= tau) {
                dtD = dtG;
                dtS = 0.0;
            } else {
                dtD = (tau / dtc) * dtG;
                dtS = dtG - dtD;
            }
            pr = -expm1(-dtS / tau);
        }
        // Eq. 32 heat flux (needed by the Shakhov target only)
        if constexpr (sizeof(P) == 4) {
            if (__any(pr > 0.0 && nn >= 3)) peculiar(pr > 0.0 && nn >= 3);
        }
        double Q[3] = {0.0, 0.0, 0.0};
        if (work && nn >= 3 && vol > 0.0 && (sizeof(P) == 8 || pr > 0.0)) {
            const double nd = (double)nn * cs.F_N / vol;
            const double f = nd * (double)nn / ((double)(nn - 1) * (double)(nn - 2));
            for (int a = 0; a < 3; ++a) Q[a] = f * 0.5 * gas.m * s2[1 + a];
            if (!isfinite(Q[0] + Q[1] + Q[2])) raise_error(G, kErrNumeric);
        }
        long long ncol = 0;
        double a_max = 0.0;
        if (active) {
            if (pr > 0.0) {
                const double qm = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
                a_max = 1.0 + 20.0 * (1.0 - gas.Pr) * qm / (p * sqrt(gas.R * T));
            }
            const double M = 0.5 * (double)nn * (double)(nn - 1) * cs.F_N * scm * dtD / vol;
            const double Mu = M + unid(draw(cs, kStreamCell, (uint64_t)(g - cs.cell0), st, 0).x);
            if (Mu >= 0.0 && Mu < 1e9) ncol = (long long)floor(Mu);
            else raise_error(G, kErrNumeric);
        }
        if (lead) {
            if (nn > 0) {                 // the tile kernel reads no record of an empty cell
                double *R = C.cellrec + (size_t)kRecLen * g;
                R[kRecU + 0] = U[0];
                R[kRecU + 1] = U[1];
                R[kRecU + 2] = U[2];
                R[kRecT] = T;
                R[kRecPr] = pr;
                R[kRecScm] = scm;
                R[kRecNcol] = (double)ncol;
                R[kRecAct] = active ? 1.0 : 0.0;
                if (pr > 0.0) {
                    R[kRecPar + 0] = Q[0];
                    R[kRecPar + 1] = Q[1];
                    R[kRecPar + 2] = Q[2];
                    R[kRecPar + 3] = p;
                    R[kRecPar + 4] = gas.R * T;
                    R[kRecPar + 5] = sqrt(2.0 * gas.R * T);
                    R[kRecPar + 6] = a_max;
                }
            }
            if (tr) {
                *tr = TraceDev{};
                tr->n = nn;
                for (int a = 0; a < 4; ++a) tr->pre_sum[a] = s1[a];
                if (active) {
                    tr->T = T;
                    tr->tau = tau;
                    tr->dt_dsmc = dtD;
                    tr->p_relax = pr;
                    tr->a_max = pr > 0.0 ? a_max : 0.0;
                }
            }
        }
    }
    tally_add<1>(C, tally, my_case, HS_CNT_SKIPPED_CELLS, skipped);
    tally_flush<1>(C, tally, HS_CNT_SKIPPED_CELLS);
    wave_flush_dtmin(C, my_case, dtmin);
}

// Steps (4)-(5) of the tiles' cells on the sorted state: NTC, SP-Shakhov resampling, Eq. 19
// rescale and sampling, with the velocities of the tile's cells (contiguous in the new
// state) staged in LDS and the cell scalars from k_cell_scalars.  Cells are served by lane
// groups as in k_cell_scalars; after the NTC every lane reads and writes only its own
// particles.
template <typename P, int TW, int D>
__device__ __forceinline__ void collide_tile_body(const Ctx &C)
{
    constexpr int MAXC = TW / 4;
    constexpr int MAXP = TW + D;
    constexpr int MAXK = 128;             // NTC candidates per chunk (two per lane)
    static_assert(MAXC <= 64, "one lane per cell at least");
    // claim word per particle slot: (round << 8) | (255 - candidate), rounds numbered across
    // the whole launch, so words of earlier rounds always lose an atomicMax of this round
    __shared__ uint32_t s_claim[MAXP];
    __shared__ P s_v[3][MAXP];
    __shared__ int32_t c_start[MAXC], c_off[MAXC + 1], c_kb[MAXC + 1];
    __shared__ P c_scm[MAXC];
    // largest sigma c seen (bits of a non-negative P: integer order = value order) and the
    // XOR hash of the accepted candidates (its low 32 bits in FP32-mixed)
    using UWord = std::conditional_t<sizeof(P) == 8, unsigned long long, unsigned int>;
    __shared__ UWord c_obs[MAXC], c_hash[MAXC];
    __shared__ int32_t c_nacc[MAXC];
    __shared__ uint8_t c_goff[MAXC], c_gkb[MAXC];
    __shared__ uint8_t s_gcell[64];       // tile-local cell of each lane's group (0xFF: none)
    Globals *G = C.g;
    if (G->halt) return;
    const int lane = threadIdx.x;
    for (int s = lane; s < MAXP; s += 64) s_claim[s] = 0u;
    uint32_t round = 0;
    const int64_t step = G->step;
    const uint32_t st = (uint32_t)step;
    const Parts<P> Dd(C.buf[(step & 1) ^ 1]);
    const int ntiles = G->n_tiles;
    const int NC = C.ncells_total;
    const GasDev &gas = C.gas;
    const bool tracing = C.trace != nullptr;
    // counts of this wave: candidates, accepted, relaxed, AR attempts, AR cap hits
    int cnt[5] = {0, 0, 0, 0, 0};        // per lane and case: small, widened when tallied
    CaseTally tally{0, -1, 0};
    int my_case = -1;

    const int xcd = blockIdx.x % kXcds, nbx = gridDim.x / kXcds;
    int pos = blockIdx.x / kXcds;
    int t = xcd_tile(pos, xcd);
    TileRef nx = tile_ref(C, t, ntiles);
    while (t < ntiles) {
        const TileRef cur = nx;
        pos += nbx;
        t = xcd_tile(pos, xcd);
        nx = tile_ref(C, t, ntiles);
        const int cb = cur.cb;
        const int ncl = cur.ce - cb;
        const int cid = cur.ci;
        if (ncl < 0 || ncl > MAXC || cb < 0 || cb + ncl > NC || cid < 0 || cid >= C.n_cases) {
            if (lane == 0) raise_error(G, kErrState);
            return;
        }
        if (ncl == 0) continue;          // a tile inside one dense cell
        if (cid != my_case) {
            const long long w5[5] = {cnt[0], cnt[1], cnt[2], cnt[3], cnt[4]};
            tally_add<5>(C, tally, my_case, HS_CNT_CANDIDATES, w5);
#pragma unroll
            for (int j = 0; j < 5; ++j) cnt[j] = 0;
            my_case = cid;
        }
        // the tile's case (uniform): RNG key, first cell, sampling on or off
        const CaseDev &cs = case_const(C, cid);
        const uint32_t sd0 = cs.seed_lo, sd1 = cs.seed_hi;
        const int lc0 = cb - cs.cell0;
        const bool samp_on = step >= cs.n_steady;
        // cell table: lane = local cell
        int nn0 = 0, n_lane = 0, start_l = 0;
        if (lane < ncl) {
            const int g0 = cb + lane;
            start_l = C.cstart[g0];
            n_lane = C.cstart[g0 + 1] - start_l;
            c_start[lane] = start_l;
            nn0 = n_lane > D ? 0 : n_lane;
        }
        const int incl = wave_incl_scan(nn0);
        const int np = __shfl(incl, 63, 64);
        if (np == 0) continue;           // empty cells only (or dense ones, served elsewhere)
        // without a dense cell the tile's slots are the contiguous run of the sorted state that
        // starts at its first cell (nearly every tile); else a slot's cell is searched for
        const bool contig = !__any(lane < ncl && n_lane > D);
        const int base0 = __shfl(start_l, 0, 64);
        if (lane < ncl) c_off[lane] = incl - nn0;
        if (lane == 0) c_off[ncl] = np;
        team_sync<64>();
        // velocities of the sorted state (written by k_sort_gather), all loads issued before
        // the first is used; FP32 words go straight from memory into LDS
        {
            constexpr int R = (MAXP + 63) / 64;
            if constexpr (sizeof(P) == 4) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int s = lane + 64 * r;
                    if (s < np) {
                        uint32_t i = (uint32_t)(base0 + s);
                        if (!contig) {
                            int a = 0, b = ncl - 1;
                            while (a < b) {
                                const int mid = (a + b + 1) >> 1;
                                if (c_off[mid] <= s) a = mid;
                                else b = mid - 1;
                            }
                            i = (uint32_t)(c_start[a] + (s - c_off[a]));
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            __builtin_amdgcn_global_load_lds((const void *)(Dd.vel[c] + i),
                                                             (__attribute__((address_space(3))) void *)&s_v[c][64 * r],
                                                             4, 0, 0);
                    }
                }
            } else {
                uint32_t boff[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int s = lane + 64 * r;
                    boff[r] = 0;
                    if (s < np) {
                        int i = base0 + s;
                        if (!contig) {
                            int a = 0, b = ncl - 1;
                            while (a < b) {
                                const int mid = (a + b + 1) >> 1;
                                if (c_off[mid] <= s) a = mid;
                                else b = mid - 1;
                            }
                            i = c_start[a] + (s - c_off[a]);
                        }
                        boff[r] = (uint32_t)i * (uint32_t)sizeof(P);
                    }
                }
                P gv[R][3];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (lane + 64 * r < np) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) gv[r][c] = ld_off(Dd.vel[c], boff[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int s = lane + 64 * r;
                    if (s < np) {
                        s_v[0][s] = gv[r][0];
                        s_v[1][s] = gv[r][1];
                        s_v[2][s] = gv[r][2];
                    }
                }
            }
        }
        // ---- lane groups sized to the work: a cell with nn particles of the tile's np gets an
        // aligned group of 2^kb ~ 64 nn / np lanes (one at least if nn > 0, none for an empty
        // or dense cell); groups are laid out largest first, which aligns each to its size
        int gsz = 0;
        if (lane < ncl) {
            const int nnc = c_off[lane + 1] - c_off[lane];
            if (nnc > 0) gsz = 1 << (31 - __clz(max(1, (64 * nnc) / np)));
        }
        for (;;) {                        // fit into 64 lanes: halve the largest group
            int tot = gsz, mx = gsz;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                tot += __shfl_xor(tot, off, 64);
                mx = max(mx, __shfl_xor(mx, off, 64));
            }
            if (tot <= 64) break;
            const unsigned long long m = __ballot(gsz == mx);
            if (lane == __ffsll((long long)m) - 1) gsz >>= 1;
        }
        {
            int goff = 0, gbase = 0;
            for (int sz = 64; sz >= 1; sz >>= 1) {
                const unsigned long long m = __ballot(gsz == sz);
                if (gsz == sz) goff = gbase + __popcll(m & ((1ull << lane) - 1ull)) * sz;
                gbase += __popcll(m) * sz;
            }
            s_gcell[lane] = 0xFF;
            team_sync<64>();
            for (int j = 0; j < gsz; ++j) s_gcell[goff + j] = (uint8_t)lane;
            if (lane < ncl) {
                c_goff[lane] = (uint8_t)(gsz > 0 ? goff : 0xFF);   // 0xFF: no group
                c_gkb[lane] = (uint8_t)(gsz > 0 ? 31 - __clz(gsz) : 0);
                c_kb[lane] = 0;
            }
            team_sync<64>();
        }
        const int gcell = s_gcell[lane];
        const bool own = gcell != 0xFF;
        const int gc = own ? gcell : 0;
        const int kb = own ? (int)c_gkb[gc] : 0;
        const int kk = 1 << kb;
        const int sub = own ? lane - (int)c_goff[gc] : 0;
        const int g = cb + gc;
        int kbmax = kb;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) kbmax = max(kbmax, __shfl_xor(kbmax, off, 64));
        double scmax = 0.0, U[3] = {0.0, 0.0, 0.0}, T = 0.0, pr = 0.0;
        P par[7] = {(P)0, (P)0, (P)0, (P)0, (P)0, (P)0, (P)0};
        int ncol = 0;
        bool active = false;
        if (own) {
            const double *R = C.cellrec + (size_t)kRecLen * g;
            scmax = R[kRecScm];
            ncol = (int)R[kRecNcol];
            active = R[kRecAct] != 0.0;
            U[0] = R[kRecU + 0];
            U[1] = R[kRecU + 1];
            U[2] = R[kRecU + 2];
            T = R[kRecT];
            pr = R[kRecPr];
            // the Shakhov parameters hold only where pr > 0 (same cache lines as the rest)
#pragma unroll
            for (int j = 0; j < 7; ++j) par[j] = (P)R[kRecPar + j];
            if (!(pr > 0.0)) {
#pragma unroll
                for (int j = 0; j < 7; ++j) par[j] = (P)0;
            }
        }
        // the velocities (FP32: still landing in LDS) and the records have arrived
        if constexpr (sizeof(P) == 4) __builtin_amdgcn_s_waitcnt(0x0F70);    // vmcnt(0)
        team_sync<64>();
        const int cn = __shfl(n_lane, gc & 63, 64);
        const bool work = own && cn <= D;
        if (!work) {
            active = false;
            ncol = 0;
            pr = 0.0;
        }
        const bool lead = work && sub == 0;

        // candidate ranges of the cells, in cell order
        if (lead) c_kb[gc] = (int)ncol;
        if (lane < ncl) {
            c_obs[lane] = 0;
            c_hash[lane] = 0;
            c_nacc[lane] = 0;
        }
        if (sub == 0 && own) c_scm[gc] = (P)scmax;
        team_sync<64>();
        const int nc_l = lane < ncl ? c_kb[lane] : 0;
        const int kincl = wave_incl_scan(nc_l);
        const int kall = __shfl(kincl, 63, 64);
        team_sync<64>();
        if (lane < ncl) c_kb[lane] = kincl - nc_l;
        if (lane == 0) c_kb[ncl] = kall;
        team_sync<64>();

        // ---- NTC (Eq. 5-9).  The candidates of a chunk are prepared by all lanes (two per
        // lane, kept in registers).  Then, in rounds, every pending candidate that is the
        // lowest-numbered pending user of both its particles is processed: such candidates
        // share no particle with each other or with an earlier pending candidate, so the
        // outcome equals the sequential order of Eq. 5-9.  (sigma c)_max is fixed during the
        // step.
        const P K_vhs = (P)gas.K_vhs, ex_vhs = (P)gas.vhs_exp;
        for (int kbase = 0; kbase < kall; kbase += MAXK) {
            const int kn = min(MAXK, kall - kbase);
            int ci[2], cj[2], clc[2], ck[2];
            P cu[2], om[2][3];
            bool pend[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int q = lane + 64 * r;
                pend[r] = q < kn;
                ci[r] = cj[r] = clc[r] = ck[r] = 0;
                cu[r] = om[r][0] = om[r][1] = om[r][2] = (P)0;
                if (pend[r]) {
                    const int x = kbase + q;
                    int a = 0, b = ncl - 1;
                    while (a < b) {
                        const int mid = (a + b + 1) >> 1;
                        if (c_kb[mid] <= x) a = mid;
                        else b = mid - 1;
                    }
                    const int kc = x - c_kb[a];
                    const int o2 = c_off[a], cn = c_off[a + 1] - o2;
                    const uint32_t lcid = (uint32_t)(lc0 + a);
                    const W4 w = draw_s(sd0, sd1, kStreamCell, lcid, st, (uint32_t)(1 + 2 * kc));
                    const uint32_t i = unidx(w.x, (uint32_t)cn);
                    uint32_t j = unidx(w.y, (uint32_t)(cn - 1));
                    if (j >= i) ++j;
                    ci[r] = o2 + (int)i;
                    cj[r] = o2 + (int)j;
                    clc[r] = a;
                    ck[r] = kc;
                    cu[r] = Real<P>::uni(w.z);
                    const W4 w2 = draw_s(sd0, sd1, kStreamCell, lcid, st, (uint32_t)(2 + 2 * kc));
                    const P cchi = (P)2 * Real<P>::uni(w2.x) - (P)1;
                    const P schi = Real<P>::sq((P)1 - cchi * cchi);
                    P sth, cth;
                    Real<P>::sc2pi(Real<P>::uni(w2.y), &sth, &cth);
                    om[r][0] = cchi;
                    om[r][1] = schi * cth;
                    om[r][2] = schi * sth;
                }
            }
            for (;;) {
                if (!__any(pend[0] || pend[1])) break;
                if (round == 0xffffffu) {          // round counter exhausted: clear the claims
                    team_sync<64>();
                    for (int s2 = lane; s2 < MAXP; s2 += 64) s_claim[s2] = 0u;
                    round = 0;
                    team_sync<64>();
                }
                ++round;
                uint32_t tag[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    tag[r] = (round << 8) | (uint32_t)(255 - (lane + 64 * r));
                    if (pend[r]) {
                        atomicMax(&s_claim[ci[r]], tag[r]);
                        atomicMax(&s_claim[cj[r]], tag[r]);
                    }
                }
                team_sync<64>();
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    if (!pend[r]) continue;
                    const int i = ci[r], j = cj[r];
                    if (s_claim[i] != tag[r] || s_claim[j] != tag[r]) continue;
                    pend[r] = false;
                    const int lc = clc[r];
                    P *vx = s_v[0], *vy = s_v[1], *vz = s_v[2];
                    const P gx = vx[i] - vx[j], gy = vy[i] - vy[j], gz = vz[i] - vz[j];
                    const P cr = Real<P>::sq(gx * gx + gy * gy + gz * gz);
                    P sc;
                    if constexpr (sizeof(P) == 4)
                        sc = cr > (P)0 ? K_vhs * __builtin_amdgcn_exp2f(ex_vhs * __builtin_amdgcn_logf(cr)) : (P)0;
                    else
                        sc = gas.K_vhs * pow(cr, gas.vhs_exp);
                    if constexpr (sizeof(P) == 8)
                        atomicMax(&c_obs[lc], (unsigned long long)__double_as_longlong(sc));
                    else
                        atomicMax(&c_obs[lc], __float_as_uint(sc));
                    if (cu[r] < sc / c_scm[lc]) {
                        const P sx = vx[i] + vx[j], sy = vy[i] + vy[j], sz = vz[i] + vz[j];
                        vx[i] = (P)0.5 * (sx - cr * om[r][0]);
                        vx[j] = (P)0.5 * (sx + cr * om[r][0]);
                        vy[i] = (P)0.5 * (sy - cr * om[r][1]);
                        vy[j] = (P)0.5 * (sy + cr * om[r][1]);
                        vz[i] = (P)0.5 * (sz - cr * om[r][2]);
                        vz[j] = (P)0.5 * (sz + cr * om[r][2]);
                        atomicAdd(&c_nacc[lc], 1);
                        atomicXor(&c_hash[lc], (UWord)((unsigned long long)(ck[r] + 1) * 0x9E3779B97F4A7C15ull));
                    }
                }
                team_sync<64>();
            }
        }
        team_sync<64>();
        if (lead && active) {
            double obs;
            if constexpr (sizeof(P) == 8) obs = __longlong_as_double((long long)c_obs[gc]);
            else obs = (double)__uint_as_float(c_obs[gc]);
            if (obs > scmax) C.sigc[g] = obs;
            cnt[0] += ncol;
            cnt[1] += c_nacc[gc];
            if (tracing) {
                TraceDev *tr = &C.trace[g];
                tr->ncol = ncol;
                tr->nacc = c_nacc[gc];
                tr->acc_hash = (unsigned long long)c_hash[gc];
            }
        }

        const int o = work ? c_off[gc] : 0;
        const int nn = work ? c_off[gc + 1] - o : 0;

        // SP-Shakhov relaxation (Eq. 16-18).  First the Bernoulli decisions of the lane's
        // particles (ids fetched four at a time) into a bit mask, then the acceptance-rejection
        // draws of the relaxing ones only, so a wave runs as many draw sequences as its
        // busiest lane has relaxing particles.
        int rel0 = 0, rel1 = 0, rel2 = 0;
        if (pr > 0.0) {
            const uint32_t *ids = Dd.id + c_start[gc];
            const int64_t nid = G->next_id[cid];
#pragma unroll 1
            for (int base = sub; base < nn; base += 64 * kk) {
                const int lim = min(nn, base + 64 * kk);
                unsigned long long mask = 0ull;
#pragma unroll 1
                for (int i0 = base; i0 < lim; i0 += 4 * kk) {
                    int64_t idv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 + u * kk;
                        idv[u] = i < lim ? full_id(ids[i], nid) : 0;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 + u * kk;
                        if (i < lim && unid(draw_s(sd0, sd1, kStreamParticle, (uint64_t)idv[u], st, kDrawRelax).x) < pr)
                            mask |= 1ull << ((i - base) / kk);
                    }
                }
                while (mask) {
                    const int bit = __ffsll((long long)mask) - 1;
                    mask &= mask - 1ull;
                    const int i = base + bit * kk;
                    const int64_t id = full_id(ids[i], nid);
                    P Cv[3];
                    int used = shakhov_draw<P>(sd0, sd1, id, st, par, (P)(1.0 - gas.Pr), Cv);
                    if (used < 0) {
                        ++rel2;
                        used = -used;
                    }
                    s_v[0][o + i] = (P)(U[0] + (double)Cv[0]);
                    s_v[1][o + i] = (P)(U[1] + (double)Cv[1]);
                    s_v[2][o + i] = (P)(U[2] + (double)Cv[2]);
                    ++rel0;
                    rel1 += used;
                }
            }
        }
        cnt[2] += rel0;
        cnt[3] += rel1;
        cnt[4] += rel2;

        // Eq. 19 rescale to the Step (3) U and T.  FP32-mixed: one pass of FP64 sums of c and
        // |c|^2 over the FP32 velocities (the peculiar sum as their difference, whose rounding
        // stays far below the FP32 storage rounding); FP64: mean first, then the peculiar sum.
        double Up[3] = {0.0, 0.0, 0.0};
        double f = 0.0;
        if constexpr (sizeof(P) == 4) {
            double r1[4] = {0.0, 0.0, 0.0, 0.0};
            if (active) {
                for (int i = sub; i < nn; i += kk) {
#pragma clang fp contract(fast)
                    const double x = (double)s_v[0][o + i], y = (double)s_v[1][o + i], z = (double)s_v[2][o + i];
                    r1[0] = r1[0] + x;
                    r1[1] = r1[1] + y;
                    r1[2] = r1[2] + z;
                    r1[3] = r1[3] + (x * x + y * y + z * z);
                }
            }
            group_sum_v<4>(r1, kb, kbmax);
            if (active) {
#pragma unroll
                for (int a = 0; a < 3; ++a) Up[a] = r1[a] / (double)nn;
                const double Tp = gas.m * (r1[3] - (r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]) / (double)nn) /
                                  (3.0 * kKB * (double)(nn - 1));
                f = Tp > 0.0 ? sqrt(T / Tp) : 0.0;
            }
        } else {
            double r1[3] = {0.0, 0.0, 0.0};
            if (active) {
                for (int i = sub; i < nn; i += kk) {
#pragma clang fp contract(fast)
                    r1[0] = r1[0] + (double)s_v[0][o + i];
                    r1[1] = r1[1] + (double)s_v[1][o + i];
                    r1[2] = r1[2] + (double)s_v[2][o + i];
                }
            }
            group_sum_v<3>(r1, kb, kbmax);
            double r2[1] = {0.0};
            if (active) {
#pragma unroll
                for (int a = 0; a < 3; ++a) Up[a] = r1[a] / (double)nn;
                for (int i = sub; i < nn; i += kk) {
#pragma clang fp contract(fast)
                    const double cx = (double)s_v[0][o + i] - Up[0], cy = (double)s_v[1][o + i] - Up[1], cz = (double)s_v[2][o + i] - Up[2];
                    r2[0] = r2[0] + (cx * cx + cy * cy + cz * cz);
                }
            }
            group_sum_v<1>(r2, kb, kbmax);
            if (active) {
                const double Tp = gas.m * r2[0] / (3.0 * kKB * (double)(nn - 1));
                f = Tp > 0.0 ? sqrt(T / Tp) : 0.0;
            }
        }
        // apply, write the final velocities, Step (5) sums
        const bool sampling = work && samp_on;
        const bool sums = sampling || (tracing && work);
        double sm[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) sm[j] = 0.0;
        if (f > 0.0 || sums) {
            for (int i = sub; i < nn; i += kk) {
#pragma clang fp contract(fast)
                double a = (double)s_v[0][o + i], b = (double)s_v[1][o + i], c = (double)s_v[2][o + i];
                if (f > 0.0) {
                    a = U[0] + (a - Up[0]) * f;
                    b = U[1] + (b - Up[1]) * f;
                    c = U[2] + (c - Up[2]) * f;
                    const size_t d = (size_t)c_start[gc] + i;
                    Dd.vel[0][d] = (P)a;
                    Dd.vel[1][d] = (P)b;
                    Dd.vel[2][d] = (P)c;
                }
                if (sums) {
                    const double c2 = a * a + b * b + c * c;
                    sm[0] += a; sm[1] += b; sm[2] += c;
                    sm[3] += a * a; sm[4] += b * b; sm[5] += c * c;
                    sm[6] += a * b; sm[7] += a * c; sm[8] += b * c;
                    sm[9] += c2 * a; sm[10] += c2 * b; sm[11] += c2 * c;
                }
            }
        }
        int nrel[3] = {rel0, rel1, rel2};
        if (tracing) {
            // the trace record keeps the group's sums of c and |c|^2 and its relaxation counts
            double t4[4] = {sm[0], sm[1], sm[2], sm[3] + sm[4] + sm[5]};
            group_sum_v<4>(t4, kb, kbmax);
#pragma unroll
            for (int j = 0; j < 3; ++j) nrel[j] = group_sum_iv(nrel[j], kb, kbmax);
            if (lead) {
                TraceDev *tr = &C.trace[g];
                for (int j = 0; j < 4; ++j) tr->post_sum[j] = t4[j];
                tr->nrelax = nrel[0];
                tr->ar_attempts = nrel[1];
                tr->ar_cap = nrel[2];
            }
        }
        if (samp_on) {
            // Step (5) sums of the tile's cells.  Each lane leaves six partial sums at a time in
            // LDS (the velocity rows: the apply loop is done with them), a group's first lane
            // also the cell's count (row 6); lane `sub` of a group adds rows j = sub, sub + kk,
            // ... over the group's lanes in lane order.  No other thread touches these cells'
            // sums in this step, so each total goes out with one atomic add (equal to a
            // load-add-store, no value returned), in one of two orders:
            //  - few cells (wide groups): the lane sends its totals itself; the lanes of one
            //    instruction then cover a few neighbouring cells;
            //  - many cells in FP32-mixed (groups of one to a few lanes, where those adds
            //    would hit a different cell in every lane): the totals go back to the group's
            //    first slot of their rows and the wave walks the tile's block of sums (13 per
            //    cell, consecutive cells) in address order, entries 0..6 of each cell in the
            //    first half, 7..12 in the second.  Empty and dense cells (no group) are skipped.
            static_assert(7 * 64 * sizeof(double) <= sizeof(s_v), "seven rows of partial sums fit");
            double *T7 = reinterpret_cast<double *>(&s_v[0][0]);
            double *Acc = C.acc + 13 * (size_t)cb;
            const int goff = lane - sub;
            const bool spread = sizeof(P) == 4 && ncl > kSampSpread;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                team_sync<64>();
#pragma unroll
                for (int j = 0; j < 6; ++j) T7[j * 64 + lane] = sm[6 * h + j];
                if (h == 0 && work && sub == 0) {
                    if (spread) T7[6 * 64 + lane] = (double)nn;
                    else unsafeAtomicAdd(&Acc[13 * gc], (double)nn);
                }
                team_sync<64>();
                // row j of a group's slots is read and rewritten by the same lane only
                for (int j = sub; work && j < 6; j += kk) {
                    double tot = 0.0;
                    for (int l = 0; l < kk; ++l) tot = tot + T7[j * 64 + goff + l];
                    if (spread) T7[j * 64 + goff] = tot;
                    else unsafeAtomicAdd(&Acc[13 * gc + 1 + 6 * h + j], tot);
                }
                if (spread) {
                    team_sync<64>();
                    const int per = 7 - h;
                    for (int k = lane; k < per * ncl; k += 64) {
                        const int cl = k / per, e = k - cl * per;
                        const int go = c_goff[cl];
                        if (go != 0xFF) {
                            const int row = h == 1 ? e : (e == 0 ? 6 : e - 1);
                            unsafeAtomicAdd(&Acc[13 * cl + 7 * h + e], T7[row * 64 + go]);
                        }
                    }
                }
            }
        }
        team_sync<64>();
    }
    const long long w5[5] = {cnt[0], cnt[1], cnt[2], cnt[3], cnt[4]};
    tally_add<5>(C, tally, my_case, HS_CNT_CANDIDATES, w5);
    tally_flush<5>(C, tally, HS_CNT_CANDIDATES);
}

constexpr int kCapWave = 192;       // densest cell of the tile kernel
constexpr int kTileW = 256;         // tile weight: particles + 4 per cell

// FP32-mixed: registers capped for four waves per SIMD (the LDS tile allows four).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_collide_tile_f32(Ctx C)
{
    collide_tile_body<float, kTileW, kCapWave>(C);
}
__global__ __launch_bounds__(64) void k_collide_tile_f64(Ctx C)
{
    collide_tile_body<double, kTileW, kCapWave>(C);
}

// Sort `a[0..p2)` ascending in LDS with a bitonic network (p2 a power of two).
template <int NB>
__device__ __forceinline__ void bitonic_sort(int32_t *a, int p2, int tid)
{
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < p2; i += NB) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const int32_t x = a[i], y = a[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Size classes of the block-per-cell kernel (dense_class).  Cells of up to kCapBlockLds
// particles are worked on in LDS: FP32 in one launch of 256-thread blocks for classes 0 and 1
// (up to kCapBlockMax) and one for class 2 (up to kCapBlockLds, 64 KB of LDS); FP64 in
// 128-thread blocks for class 0 (the FP64 kernel needs 256 registers a lane, so a 256-thread
// block fills a compute unit alone; two 128-thread blocks per unit keep twice as many cells in
// flight) and 256-thread blocks for classes 1 and 2 (112 KB of LDS).  A denser cell (class 3)
// takes the global launch: its velocities stay in the new state's arrays and its claim words
// and sorted sources in two per-particle scratch arrays the step no longer needs at that point
// (the move's slots and new cells), so no cell of a case is too dense.  A launch visits the
// lists of its classes only; results do not depend on the class.

template <typename P, int CAPB, int NB, bool GLOB = false>
__global__ __launch_bounds__(NB) void k_collide_dense(Ctx C, int cls_lo, int cls_hi)
{
    constexpr int KC = 2 * NB;             // NTC candidates per chunk (two per thread)
    static_assert(KC <= 1024, "candidate number fits the claim word");
    constexpr int CAPL = GLOB ? 4 : CAPB;  // LDS rows (the global class keeps its cell in memory)
    __shared__ __attribute__((aligned(16))) int32_t s_src[CAPL];   // sources during the gather, then claim words
    __shared__ P s_v[3][CAPL];
    __shared__ double s_red[(NB / 64) * 12];
    __shared__ unsigned long long s_obs, s_hash;
    __shared__ int s_nacc, s_left;
    __shared__ int32_t s_rel[3];
    __shared__ int s_rows[8];                  // runs starting in each row of 64 slots (ranking)
    uint32_t *s_claim = (uint32_t *)s_src;
    Globals *G = C.g;
    if (G->halt) return;
    const int tid = threadIdx.x;
    const int64_t step = G->step;
    const uint32_t st = (uint32_t)step;
    const Parts<P> S(C.buf[step & 1]);
    const Parts<P> Dd(C.buf[(step & 1) ^ 1]);
    const bool use_perm = C.perm != nullptr;
    // the cells of size classes cls_lo .. cls_hi (at most two), one list after the other
    const int nlo = G->n_big[cls_lo];
    const int nbig = nlo + (cls_hi > cls_lo ? G->n_big[cls_hi] : 0);
    const GasDev &gas = C.gas;
    const bool tracing = C.trace != nullptr;
    CellCounts cc{0, 0, 0, 0, 0, 0};
    int my_case = -1;
    for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
        const int g = b < nlo ? C.big_list[C.big_off[cls_lo] + b] : C.big_list[C.big_off[cls_hi] + (b - nlo)];
        const int s0 = C.cstart[g];
        const int n = C.cstart[g + 1] - s0;
        const int cid = case_of(C, g);
        const CaseDev &cs = C.cases[cid];
        if (n <= C.cap_wave || (!GLOB && n > CAPB)) {   // not of this launch's classes
            if (tid == 0) raise_error(G, kErrState);
            continue;
        }
        if (tid == 0 && cid != my_case) {
            if (my_case >= 0) flush_counts(C, my_case, cc);
            my_case = cid;
        }
        // the cell's working velocities and claim words: LDS, or for the global class the new
        // state's rows of the cell and the move's slot array (dead after the scatter)
        P *sv[3];
        uint32_t *claim;
        int32_t *srt;                          // sources in stable order
        if constexpr (GLOB) {
            for (int a = 0; a < 3; ++a) sv[a] = Dd.vel[a] + s0;
            claim = reinterpret_cast<uint32_t *>(C.slot + s0);
            srt = C.newcell + s0;
        } else {
            for (int a = 0; a < 3; ++a) sv[a] = s_v[a];
            claim = s_claim;
            srt = s_src;
        }
        // stable order (sort of the source indices), gather, sorted state
        if constexpr (GLOB) {
            // rank of each source among the cell's (sources are distinct)
            for (int k = tid; k < n; k += NB) {
                const int src = use_perm ? C.perm[s0 + k] : s0 + k;
                int rk = 0;
                if (use_perm)
                    for (int j = 0; j < n; ++j) rk += (int)(C.perm[s0 + j] < src);
                else
                    rk = k;
                srt[rk] = src;
            }
        }
        // up to kRankMax particles: each source's rank among the cell's (sources are distinct)
        // from its runs: the slots split into maximal runs of increasing sources inside one
        // aligned block of 64 source indices (the move hands out a wave's slots of a cell as one
        // such run).  Runs of different blocks are ordered by their block, so a source's rank is
        // the length of the runs of lower blocks plus, in each run of its own block (its own
        // run, rarely another), the sources below it (binary search).  Run starts and blocks go
        // to the first two velocity rows and the sorted sources to the third, all free until
        // the gather.  Denser cells: bitonic sort in place.
        constexpr int kRankMax = CAPB < 512 ? CAPB : 512;
        constexpr int GRK = (kRankMax + NB - 1) / NB;
        static_assert(kRankMax / 64 <= 8, "run counts of the rows fit");
        const bool by_rank = !GLOB && use_perm && n <= kRankMax;
        int rsrc[GRK];
        if constexpr (!GLOB) {
            int p2 = 4;
            while (p2 < n) p2 <<= 1;
            for (int k = tid; k < p2; k += NB) s_src[k] = k < n ? (use_perm ? C.perm[s0 + k] : s0 + k) : 0x7fffffff;
            __syncthreads();
            if (by_rank) {
                int32_t *run_at = reinterpret_cast<int32_t *>(&s_v[0][0]);
                int32_t *run_blk = reinterpret_cast<int32_t *>(&s_v[1][0]);
                int32_t *rk_out = reinterpret_cast<int32_t *>(&s_v[2][0]);
                const int lane = tid & 63, nrow = (n + 63) >> 6;
                auto run_head = [&](int k) {
                    if (k >= n) return false;
                    if (k == 0) return true;
                    const int x = s_src[k], y = s_src[k - 1];
                    return (x >> 6) != (y >> 6) || x < y;
                };
                for (int r = tid >> 6; r < nrow; r += NB / 64) {
                    const unsigned long long m = __ballot(run_head(64 * r + lane));
                    if (lane == 0) s_rows[r] = __popcll(m);
                }
                __syncthreads();
                int nrun = 0;
                for (int r = 0; r < nrow; ++r) nrun += s_rows[r];
                for (int r = tid >> 6; r < nrow; r += NB / 64) {
                    int before = 0;
                    for (int q = 0; q < r; ++q) before += s_rows[q];
                    const int k = 64 * r + lane;
                    const bool h = run_head(k);
                    const unsigned long long m = __ballot(h);
                    if (h) {
                        const int j = before + __popcll(m & ((1ull << lane) - 1ull));
                        run_at[j] = k;
                        run_blk[j] = s_src[k] >> 6;
                    }
                }
                if (tid == 0) run_at[nrun] = n;
                __syncthreads();
                for (int k = tid; k < n; k += NB) {
                    const int x = s_src[k], bx = x >> 6;
                    int rk = 0;
                    for (int j = 0; j < nrun; ++j) {
                        const int bj = run_blk[j], a = run_at[j], e = run_at[j + 1];
                        if (bj < bx) {
                            rk += e - a;
                        } else if (bj == bx) {
                            int lo = a, hi = e;            // first source of the run not below x
                            while (lo < hi) {
                                const int mid = (lo + hi) >> 1;
                                if (s_src[mid] < x) lo = mid + 1;
                                else hi = mid;
                            }
                            rk += lo - a;
                        }
                    }
                    rk_out[rk] = x;
                }
                __syncthreads();
                // every thread takes its sources before any velocity row is written
#pragma unroll
                for (int r = 0; r < GRK; ++r) {
                    const int k = tid + NB * r;
                    rsrc[r] = k < n ? rk_out[k] : 0;
                }
            } else if (use_perm) {
                bitonic_sort<NB>(s_src, p2, tid);
            }
        }
        __syncthreads();
        auto gather_one = [&](int k, int src) {
            const size_t dst = (size_t)s0 + k;
            for (int a = 0; a < 3; ++a) if (a < cs.dim) Dd.pos[a][dst] = S.pos[a][src];
            Dd.cell[dst] = g;
            Dd.id[dst] = S.id[src];
            const P v0 = S.vel[0][src], v1 = S.vel[1][src], v2 = S.vel[2][src];
            sv[0][k] = v0;
            sv[1][k] = v1;
            sv[2][k] = v2;
        };
        if (by_rank) {
#pragma unroll
            for (int r = 0; r < GRK; ++r) {
                const int k = tid + NB * r;
                if (k < n) gather_one(k, rsrc[r]);
            }
        } else {
            for (int k = tid; k < n; k += NB) gather_one(k, srt[k]);
        }
        __syncthreads();
        for (int k = tid; k < n; k += NB) claim[k] = 0u;
        if (tid == 0) {
            s_obs = 0ull;
            s_hash = 0ull;
            s_nacc = 0;
            s_rel[0] = s_rel[1] = s_rel[2] = 0;
        }

        // Eq. 31 moments
        double s1[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = tid; k < n; k += NB) {
#pragma clang fp contract(fast)
            const double x = (double)sv[0][k], y = (double)sv[1][k], z = (double)sv[2][k];
            s1[0] = s1[0] + x;
            s1[1] = s1[1] + y;
            s1[2] = s1[2] + z;
            s1[3] = s1[3] + (x * x + y * y + z * z);
        }
        team_sum<NB, 4>(s1, s_red);
        double U[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) U[a] = s1[a] / (double)n;
        double s2[4] = {0.0, 0.0, 0.0, 0.0};
        if constexpr (sizeof(P) == 4) {
            float uf[3], ud[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                uf[a] = (float)U[a];
                ud[a] = (float)(U[a] - (double)uf[a]);
            }
            for (int k = tid; k < n; k += NB) {
#pragma clang fp contract(fast)
                const float cx = (sv[0][k] - uf[0]) - ud[0];
                const float cy = (sv[1][k] - uf[1]) - ud[1];
                const float cz = (sv[2][k] - uf[2]) - ud[2];
                const float c2 = cx * cx + cy * cy + cz * cz;
                s2[0] = s2[0] + (double)c2;
                s2[1] = s2[1] + (double)(c2 * cx);
                s2[2] = s2[2] + (double)(c2 * cy);
                s2[3] = s2[3] + (double)(c2 * cz);
            }
        } else {
            for (int k = tid; k < n; k += NB) {
#pragma clang fp contract(fast)
                const double cx = sv[0][k] - U[0], cy = sv[1][k] - U[1], cz = sv[2][k] - U[2];
                const double c2 = cx * cx + cy * cy + cz * cz;
                s2[0] = s2[0] + c2;
                s2[1] = s2[1] + c2 * cx;
                s2[2] = s2[2] + c2 * cy;
                s2[3] = s2[3] + c2 * cz;
            }
        }
        team_sum<NB, 4>(s2, s_red);

        // Eq. 10 / 25-28 split, N_col, Shakhov parameters (every thread alike)
        TraceDev *tr = (tid == 0 && tracing) ? &C.trace[g] : nullptr;
        const double vol = C.vol[g];
        double T;
        if constexpr (sizeof(P) == 4)
            T = gas.m * (s1[3] - (s1[0] * s1[0] + s1[1] * s1[1] + s1[2] * s1[2]) / (double)n) /
                (3.0 * kKB * (double)(n - 1));
        else
            T = gas.m * s2[0] / (3.0 * kKB * (double)(n - 1));
        double Q[3] = {0.0, 0.0, 0.0};
        if (vol > 0.0) {
            const double nd = (double)n * cs.F_N / vol;
            const double f = nd * (double)n / ((double)(n - 1) * (double)(n - 2));
            for (int a = 0; a < 3; ++a) Q[a] = f * 0.5 * gas.m * s2[1 + a];
        }
        if (tid == 0 && (!isfinite(T) || !isfinite(Q[0] + Q[1] + Q[2]))) raise_error(G, kErrNumeric);
        const bool active = T > 0.0 && vol > 0.0;
        if (tr) {
            *tr = TraceDev{};
            tr->n = n;
            for (int a = 0; a < 4; ++a) tr->pre_sum[a] = s1[a];
        }
        double pr = 0.0, scmax = 0.0;
        long long ncol = 0;
        P par[7] = {(P)0, (P)0, (P)0, (P)0, (P)0, (P)0, (P)0};
        if (!active) {
            if (tid == 0) cc.skipped++;
        } else {
            const double nd = (double)n * cs.F_N / vol;
            const double p = nd * kKB * T;
            const double tau = gas.mu_ref * pow(T / gas.T_ref, gas.omega) / p;
            const double dtG = cs.dim == 0 ? C.dt_cell[g] : G->dt_cur[cid];
            double dtc;
            if (cs.dim == 0) {
                dtc = dtG;
            } else {
                const double um = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
                dtc = (cs.mesh ? C.mgeo[2 * (size_t)g + 1] : cs.L_cell) / (um + sqrt(gas.gamma * gas.R * T));
                // Eq. 26: the next global step is the smallest local step of this one
                if (cs.adapt_dt && tid == 0)
                    atomicMin(&G->dt_next[cid], (unsigned long long)__double_as_longlong(dtc));
            }
            double dtD, dtS;
            if (dtc <= tau) {
                dtD = dtG;
                dtS = 0.0;
            } else {
                dtD = (tau / dtc) * dtG;
                dtS = dtG - dtD;
            }
            pr = -expm1(-dtS / tau);
            double a_max = 1.0;
            if (pr > 0.0) {
                const double qm = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
                a_max = 1.0 + 20.0 * (1.0 - gas.Pr) * qm / (p * sqrt(gas.R * T));
                par[0] = (P)Q[0];
                par[1] = (P)Q[1];
                par[2] = (P)Q[2];
                par[3] = (P)p;
                par[4] = (P)(gas.R * T);
                par[5] = (P)sqrt(2.0 * gas.R * T);
                par[6] = (P)a_max;
            }
            scmax = C.sigc[g];
            const double M = 0.5 * (double)n * (double)(n - 1) * cs.F_N * scmax * dtD / vol;
            const double Mu = M + unid(draw(cs, kStreamCell, (uint64_t)(g - cs.cell0), st, 0).x);
            if (Mu >= 0.0 && Mu < 1e9) ncol = (long long)floor(Mu);
            else if (tid == 0) raise_error(G, kErrNumeric);
            if (tr) {
                tr->T = T;
                tr->tau = tau;
                tr->dt_dsmc = dtD;
                tr->p_relax = pr;
                tr->a_max = pr > 0.0 ? a_max : 0.0;
            }
        }
        __syncthreads();

        // NTC (Eq. 5-9) in rounds over the block, as in k_collide_tile
        const uint32_t lc = (uint32_t)(g - cs.cell0);
        const P scm = (P)scmax;
        uint32_t round = 0;
        for (long long kbase = 0; kbase < ncol; kbase += KC) {
            const int kn = (int)min((long long)KC, ncol - kbase);
            int ci[2], cj[2];
            long long ck[2];
            P cu[2], om[2][3];
            bool pend[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int q = tid + NB * r;
                pend[r] = q < kn;
                ci[r] = cj[r] = 0;
                ck[r] = 0;
                cu[r] = om[r][0] = om[r][1] = om[r][2] = (P)0;
                if (pend[r]) {
                    const long long kc = kbase + q;
                    const W4 w = draw(cs, kStreamCell, lc, st, (uint32_t)(1 + 2 * kc));
                    const uint32_t i = unidx(w.x, (uint32_t)n);
                    uint32_t j = unidx(w.y, (uint32_t)(n - 1));
                    if (j >= i) ++j;
                    ci[r] = (int)i;
                    cj[r] = (int)j;
                    ck[r] = kc;
                    cu[r] = Real<P>::uni(w.z);
                    const W4 w2 = draw(cs, kStreamCell, lc, st, (uint32_t)(2 + 2 * kc));
                    const P cchi = (P)2 * Real<P>::uni(w2.x) - (P)1;
                    const P schi = Real<P>::sq((P)1 - cchi * cchi);
                    P sth, cth;
                    Real<P>::sc2pi(Real<P>::uni(w2.y), &sth, &cth);
                    om[r][0] = cchi;
                    om[r][1] = schi * cth;
                    om[r][2] = schi * sth;
                }
            }
            __syncthreads();                   // every thread has left the previous chunk's rounds
            if (tid == 0) s_left = kn;
            __syncthreads();
            for (;;) {
                if (round == 0x3fffffu) {      // round counter exhausted: clear the claims
                    for (int k = tid; k < n; k += NB) claim[k] = 0u;
                    round = 0;
                    __syncthreads();
                }
                ++round;
                uint32_t tag[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    tag[r] = (round << 10) | (uint32_t)(1023 - (tid + NB * r));
                    if (pend[r]) {
                        atomicMax(&claim[ci[r]], tag[r]);
                        atomicMax(&claim[cj[r]], tag[r]);
                    }
                }
                __syncthreads();
                int done = 0;
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    if (!pend[r]) continue;
                    const int i = ci[r], j = cj[r];
                    if (claim[i] != tag[r] || claim[j] != tag[r]) continue;
                    pend[r] = false;
                    ++done;
                    P *vx = sv[0], *vy = sv[1], *vz = sv[2];
                    const P gx = vx[i] - vx[j], gy = vy[i] - vy[j], gz = vz[i] - vz[j];
                    const P cr = Real<P>::sq(gx * gx + gy * gy + gz * gz);
                    P sc;
                    if constexpr (sizeof(P) == 4)
                        sc = cr > (P)0 ? (P)gas.K_vhs * __builtin_amdgcn_exp2f((P)gas.vhs_exp * __builtin_amdgcn_logf(cr))
                                       : (P)0;
                    else
                        sc = gas.K_vhs * pow(cr, gas.vhs_exp);
                    atomicMax(&s_obs, (unsigned long long)__double_as_longlong((double)sc));
                    if (cu[r] < sc / scm) {
                        const P sx = vx[i] + vx[j], sy = vy[i] + vy[j], sz = vz[i] + vz[j];
                        vx[i] = (P)0.5 * (sx - cr * om[r][0]);
                        vx[j] = (P)0.5 * (sx + cr * om[r][0]);
                        vy[i] = (P)0.5 * (sy - cr * om[r][1]);
                        vy[j] = (P)0.5 * (sy + cr * om[r][1]);
                        vz[i] = (P)0.5 * (sz - cr * om[r][2]);
                        vz[j] = (P)0.5 * (sz + cr * om[r][2]);
                        atomicAdd(&s_nacc, 1);
                        atomicXor(&s_hash, (unsigned long long)(ck[r] + 1) * 0x9E3779B97F4A7C15ull);
                    }
                }
                if (done) atomicSub(&s_left, done);
                __syncthreads();
                if (s_left == 0) break;
            }
        }
        if (tid == 0 && active) {
            const double obs = __longlong_as_double((long long)s_obs);
            if (obs > scmax) C.sigc[g] = obs;
            cc.cand += ncol;
            cc.acc += s_nacc;
            if (tr) {
                tr->ncol = ncol;
                tr->nacc = s_nacc;
                tr->acc_hash = s_hash;
            }
        }

        // SP-Shakhov relaxation (Eq. 16-18)
        if (pr > 0.0) {
            int nrel = 0, nar = 0, ncap = 0;
            // decisions first (32 particles per thread at a time), then the draws
            for (int k0 = tid; k0 < n; k0 += 32 * NB) {
            uint32_t mask = 0u;
            for (int k = k0, j = 0; k < n && j < 32; k += NB, ++j) {
                const int64_t id = full_id(Dd.id[(size_t)s0 + k], G->next_id[cid]);
                if (unid(draw(cs, kStreamParticle, (uint64_t)id, st, kDrawRelax).x) < pr) mask |= 1u << j;
            }
            while (mask) {
                const int j = __ffs((int)mask) - 1;
                mask &= mask - 1u;
                const int k = k0 + NB * j;
                const int64_t id = full_id(Dd.id[(size_t)s0 + k], G->next_id[cid]);
                P Cv[3];
                int used = shakhov_draw<P>(cs.seed_lo, cs.seed_hi, id, st, par, (P)(1.0 - gas.Pr), Cv);
                if (used < 0) {
                    ++ncap;
                    used = -used;
                }
                ++nrel;
                nar += used;
                sv[0][k] = (P)(U[0] + (double)Cv[0]);
                sv[1][k] = (P)(U[1] + (double)Cv[1]);
                sv[2][k] = (P)(U[2] + (double)Cv[2]);
            }
            }
            if (nrel) atomicAdd(&s_rel[0], nrel);
            if (nar) atomicAdd(&s_rel[1], nar);
            if (ncap) atomicAdd(&s_rel[2], ncap);
        }
        __syncthreads();

        // Eq. 19 rescale (each thread rescales the particles it summed), Step (5) sums
        double r1[3] = {0.0, 0.0, 0.0};
        for (int k = tid; k < n; k += NB) {
#pragma clang fp contract(fast)
            r1[0] = r1[0] + (double)sv[0][k];
            r1[1] = r1[1] + (double)sv[1][k];
            r1[2] = r1[2] + (double)sv[2][k];
        }
        team_sum<NB, 3>(r1, s_red);
        const double Up[3] = {r1[0] / (double)n, r1[1] / (double)n, r1[2] / (double)n};
        double r2[1] = {0.0};
        for (int k = tid; k < n; k += NB) {
#pragma clang fp contract(fast)
            const double cx = (double)sv[0][k] - Up[0], cy = (double)sv[1][k] - Up[1], cz = (double)sv[2][k] - Up[2];
            r2[0] = r2[0] + (cx * cx + cy * cy + cz * cz);
        }
        team_sum<NB, 1>(r2, s_red);
        double f = 0.0;
        if (active) {
            const double Tp = gas.m * r2[0] / (3.0 * kKB * (double)(n - 1));
            f = Tp > 0.0 ? sqrt(T / Tp) : 0.0;
        }
        const bool sampling = step >= cs.n_steady;
        const bool sums = sampling || tracing;
        double sm[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) sm[j] = 0.0;
        for (int k = tid; k < n; k += NB) {
#pragma clang fp contract(fast)
            double a = (double)sv[0][k], bb = (double)sv[1][k], c = (double)sv[2][k];
            if (f > 0.0) {
                a = U[0] + (a - Up[0]) * f;
                bb = U[1] + (bb - Up[1]) * f;
                c = U[2] + (c - Up[2]) * f;
            }
            const size_t dst = (size_t)s0 + k;
            Dd.vel[0][dst] = (P)a;
            Dd.vel[1][dst] = (P)bb;
            Dd.vel[2][dst] = (P)c;
            if (sums) {
                const double c2 = a * a + bb * bb + c * c;
                sm[0] += a; sm[1] += bb; sm[2] += c;
                sm[3] += a * a; sm[4] += bb * bb; sm[5] += c * c;
                sm[6] += a * bb; sm[7] += a * c; sm[8] += bb * c;
                sm[9] += c2 * a; sm[10] += c2 * bb; sm[11] += c2 * c;
            }
        }
        if (sums) team_sum<NB, 12>(sm, s_red);
        if (tid == 0) {
            cc.relax += s_rel[0];
            cc.ar += s_rel[1];
            cc.arcap += s_rel[2];
            if (sampling) {
                double *A = &C.acc[13 * (size_t)g];
                A[0] += (double)n;
#pragma unroll
                for (int j = 0; j < 12; ++j) A[1 + j] += sm[j];
            }
            if (tr) {
                tr->post_sum[0] = sm[0];
                tr->post_sum[1] = sm[1];
                tr->post_sum[2] = sm[2];
                tr->post_sum[3] = sm[3] + sm[4] + sm[5];
                tr->nrelax = s_rel[0];
                tr->ar_attempts = s_rel[1];
                tr->ar_cap = s_rel[2];
            }
        }
        __syncthreads();
    }
    if (tid == 0 && my_case >= 0) flush_counts(C, my_case, cc);
}

// Dense-cell list of a batch whose cells never re-sort (only 0-D cases): built once.
__global__ void k_build_big(Ctx C)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = g < C.ncells_total;
    const int n = in ? C.cstart[g + 1] - C.cstart[g] : 0;
    add_dense(C, g, n, in && n > C.cap_wave);
}

__global__ void k_finish_step(Ctx C, int sorted)
{
    Globals *G = C.g;
    if (G->halt) return;
    const int64_t step = G->step;
    for (int c = threadIdx.x; c < C.n_cases; c += blockDim.x) {
        const CaseDev &cs = C.cases[c];
        if (step >= cs.n_steady) {
            G->n_samples[c] += 1;
            G->t_sampled[c] = G->t_sampled[c] + G->dt_cur[c];
        }
        // Eq. 26 for the next step (kept when no cell was active)
        if (cs.adapt_dt && cs.dim > 0 && G->dt_next[c] != kInfBits) G->dt_cur[c] = __longlong_as_double((long long)G->dt_next[c]);
        G->dt_next[c] = kInfBits;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (sorted) {
            G->n_live = G->n_new;
            for (int k = 0; k < kDenseClasses; ++k) G->n_big[k] = 0;   // rebuilt by the next step's scan
        }
        G->n_work = 0;
        G->n_total = G->n_live;
        G->step = step + 1;
    }
}

// ------------------------------------------------------------------------------------
// Output (Step 6) and checks
// ------------------------------------------------------------------------------------

// Current-state Eq. 31 estimators of one case: n, U (3), T, q (3) per cell.
template <typename P>
__global__ void k_moments_now(Ctx C, int case_id, double *out)
{
    const CaseDev &cs = C.cases[case_id];
    const int lc = blockIdx.x * blockDim.x + threadIdx.x;
    if (lc >= cs.ncells) return;
    const int g = cs.cell0 + lc;
    const Parts<P> S(C.buf[C.g->step & 1]);
    const int s = C.cstart[g], n = C.cstart[g + 1] - s;
    double U[3] = {0.0, 0.0, 0.0}, T = 0.0, q[3] = {0.0, 0.0, 0.0};
    const double vol = C.vol[g];
    if (n >= 1) {
        for (int k = 0; k < n; ++k)
            for (int a = 0; a < 3; ++a) U[a] = U[a] + (double)S.vel[a][s + k];
        for (int a = 0; a < 3; ++a) U[a] = U[a] / (double)n;
    }
    if (n >= 2) {
        double s2 = 0.0, s3[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < n; ++k) {
            double c[3], c2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                c[a] = (double)S.vel[a][s + k] - U[a];
                c2 = c2 + c[a] * c[a];
            }
            s2 = s2 + c2;
            for (int a = 0; a < 3; ++a) s3[a] = s3[a] + c2 * c[a];
        }
        T = C.gas.m * s2 / (3.0 * kKB * (double)(n - 1));
        if (n >= 3 && vol > 0.0) {
            const double nd = (double)n * cs.F_N / vol;
            const double f = nd * (double)n / ((double)(n - 1) * (double)(n - 2));
            for (int a = 0; a < 3; ++a) q[a] = f * 0.5 * C.gas.m * s3[a];
        }
    }
    double *o = out + 8 * (size_t)lc;
    o[0] = vol > 0.0 ? (double)n * cs.F_N / vol : 0.0;
    o[1] = U[0];
    o[2] = U[1];
    o[3] = U[2];
    o[4] = T;
    o[5] = q[0];
    o[6] = q[1];
    o[7] = q[2];
}

// Step (6) time averages of one case from the Step (5) sums: n, U (3), T, q (3) per cell.
__global__ void k_finalize(Ctx C, int case_id, double *out)
{
    const CaseDev &cs = C.cases[case_id];
    const int lc = blockIdx.x * blockDim.x + threadIdx.x;
    if (lc >= cs.ncells) return;
    const int g = cs.cell0 + lc;
    const double *A = &C.acc[13 * (size_t)g];
    const double S = (double)C.g->n_samples[case_id];
    double nn = 0.0, U[3] = {0.0, 0.0, 0.0}, T = 0.0, q[3] = {0.0, 0.0, 0.0};
    const double vol = C.vol[g];
    if (A[0] > 0.0 && S > 0.0 && vol > 0.0) {
        nn = cs.F_N * A[0] / (S * vol);
        for (int a = 0; a < 3; ++a) U[a] = A[1 + a] / A[0];
        const double cc = (A[4] + A[5] + A[6]) / A[0];
        const double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
        T = C.gas.m / (3.0 * kKB) * (cc - uu);
        const double cij[3][3] = {{A[4], A[7], A[8]}, {A[7], A[5], A[9]}, {A[8], A[9], A[6]}};
        for (int a = 0; a < 3; ++a) {
            double uc = 0.0;
            for (int b = 0; b < 3; ++b) uc = uc + U[b] * cij[a][b] / A[0];
            q[a] = 0.5 * C.gas.m * nn * (A[10 + a] / A[0] - 2.0 * uc - U[a] * cc + 2.0 * U[a] * uu);
        }
    }
    double *o = out + 8 * (size_t)lc;
    o[0] = nn;
    o[1] = U[0];
    o[2] = U[1];
    o[3] = U[2];
    o[4] = T;
    o[5] = q[0];
    o[6] = q[1];
    o[7] = q[2];
}

__global__ void k_philox(uint64_t seed, uint32_t stream, uint64_t e0, uint32_t step, uint32_t d, int64_t n,
                         uint32_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    CaseDev cs;
    cs.seed_lo = (uint32_t)seed;
    cs.seed_hi = (uint32_t)(seed >> 32);
    const W4 w = draw(cs, stream, e0 + (uint64_t)i, step, d);
    out[4 * i + 0] = w.x;
    out[4 * i + 1] = w.y;
    out[4 * i + 2] = w.z;
    out[4 * i + 3] = w.w;
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------


static inline hipStream_t S_(void *s) { return (hipStream_t)s; }
static inline int blocks_for(long long n, int per) { return (int)((n + per - 1) / per); }
static inline int stream_grid() { return 256 * 16; }

void Launch::init_cells(const Ctx &c, void *s)
{
    hipLaunchKernelGGL(k_init_cells, dim3(blocks_for(c.ncells_total, kBlock)), dim3(kBlock), 0, S_(s), c, 1);
}
void Launch::init_count(const Ctx &c, void *s)
{
    hipLaunchKernelGGL(k_init_cells, dim3(blocks_for(c.ncells_total, kBlock)), dim3(kBlock), 0, S_(s), c, 0);
}
void Launch::init_fill(const Ctx &c, void *s)
{
    if (c.precision == HS_FP64)
        hipLaunchKernelGGL(k_init_fill<double>, dim3(blocks_for(c.ncells_total, 64)), dim3(64), 0, S_(s), c);
    else
        hipLaunchKernelGGL(k_init_fill<float>, dim3(blocks_for(c.ncells_total, 64)), dim3(64), 0, S_(s), c);
}
void Launch::init_finish(const Ctx &c, void *s)
{
    hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(256), 0, S_(s), c, (int64_t)0);
}
void Launch::tile_table(const Ctx &c, void *s)
{
    hipLaunchKernelGGL(k_case_tiles, dim3(1), dim3(kBlock), 0, S_(s), c);
    hipLaunchKernelGGL(k_tile_table, dim3((c.ncells_total + kBlock - 1) / kBlock), dim3(kBlock), 0, S_(s), c);
}

void Launch::scan_cells(const Ctx &c, void *s, int build_big)
{
    const int nparts = blocks_for(c.ncells_total, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nparts), dim3(kBlock), 0, S_(s), c);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, S_(s), c, nparts);
    hipLaunchKernelGGL(k_scan_final, dim3(nparts), dim3(kBlock), 0, S_(s), c, build_big, nparts);
    tile_table(c, s);
}
void Launch::inject(const Ctx &c, void *s)
{
    if (c.n_faces == 0) return;
    hipLaunchKernelGGL(k_inject_count, dim3(blocks_for(c.n_faces, kBlock)), dim3(kBlock), 0, S_(s), c);
    hipLaunchKernelGGL(k_inject_scan, dim3(1), dim3(1024), 0, S_(s), c);
    if (c.precision == HS_FP64)
        hipLaunchKernelGGL(k_inject_fill<double>, dim3(blocks_for(c.n_faces, 4)), dim3(kBlock), 0, S_(s), c);
    else
        hipLaunchKernelGGL(k_inject_fill<float>, dim3(blocks_for(c.n_faces, 4)), dim3(kBlock), 0, S_(s), c);
}
void Launch::move_count(const Ctx &c, void *s, int any_body)
{
    const int grid = c.grid[HS_KERNEL_MOVE] > 0 ? c.grid[HS_KERNEL_MOVE]
                                                : std::min(4 * stream_grid(), blocks_for(c.capacity, kBlock));
    // the worklist holds the body-near particles of grid cases (about 1%); mesh cases have
    // their own kernel over the whole particle array
    if (c.precision == HS_FP64) {
        hipLaunchKernelGGL(k_move_fast<double>, dim3(grid), dim3(kBlock), 0, S_(s), c);
        if (c.mxy || c.hxyz) hipLaunchKernelGGL(k_move_mesh<double>, dim3(grid), dim3(kBlock), 0, S_(s), c);
        if (any_body) hipLaunchKernelGGL(k_move_body<double>, dim3(256), dim3(kBlock), 0, S_(s), c);
    } else {
        hipLaunchKernelGGL(k_move_fast<float>, dim3(grid), dim3(kBlock), 0, S_(s), c);
        if (c.mxy || c.hxyz) hipLaunchKernelGGL(k_move_mesh<float>, dim3(grid), dim3(kBlock), 0, S_(s), c);
        if (any_body) hipLaunchKernelGGL(k_move_body<float>, dim3(256), dim3(kBlock), 0, S_(s), c);
    }
}
void Launch::scatter(const Ctx &c, void *s)
{
    const int grid = c.grid[HS_KERNEL_SCATTER] > 0 ? c.grid[HS_KERNEL_SCATTER]
                                                   : std::min(stream_grid(), blocks_for(c.capacity, kBlock));
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(kBlock), 0, S_(s), c);
}
// Tile kernels loop over tiles with a fixed grid: wide for the streaming gather and scalar
// kernels, about the resident capacity for the collision kernel (its per-wave setup and
// counter flush are paid once per block).
static int tile_grid(const Ctx &c, int which, long long cap)
{
    long long g = c.grid[which];
    if (g <= 0) {
        const long long maxtiles = ((long long)c.capacity + 4ll * c.ncells_total) / kTileW + 1;
        g = std::max(1ll, std::min(maxtiles, cap));
    }
    return (int)((g + kXcds - 1) / kXcds * kXcds);     // whole blocks per XCD
}
void Launch::gather(const Ctx &c, void *s)
{
    const int g = tile_grid(c, HS_KERNEL_GATHER, 256ll * 32);
    if (c.precision == HS_FP64) hipLaunchKernelGGL((k_sort_gather<double, kTileW, kCapWave>), dim3(g), dim3(64), 0, S_(s), c);
    else hipLaunchKernelGGL((k_sort_gather<float, kTileW, kCapWave>), dim3(g), dim3(64), 0, S_(s), c);
}
void Launch::scalars(const Ctx &c, void *s)
{
    const int g = tile_grid(c, HS_KERNEL_SCALARS, 256ll * 32);
    if (c.precision == HS_FP64) hipLaunchKernelGGL((k_cell_scalars<double, kTileW, kCapWave>), dim3(g), dim3(64), 0, S_(s), c);
    else hipLaunchKernelGGL((k_cell_scalars<float, kTileW, kCapWave>), dim3(g), dim3(64), 0, S_(s), c);
}
void Launch::collide(const Ctx &c, void *s)
{
    if (c.precision == HS_FP64)
        hipLaunchKernelGGL(k_collide_tile_f64, dim3(tile_grid(c, HS_KERNEL_COLLIDE, 256ll * 4)), dim3(64), 0, S_(s), c);
    else
        hipLaunchKernelGGL(k_collide_tile_f32, dim3(tile_grid(c, HS_KERNEL_COLLIDE, 256ll * 16)), dim3(64), 0, S_(s), c);
}
void Launch::dense(const Ctx &c, void *s)
{
    const int gb = c.grid[HS_KERNEL_DENSE] > 0 ? c.grid[HS_KERNEL_DENSE] : std::max(1, std::min(c.ncells_total, 256 * 2));
    // the two densest classes are rare: a few blocks each
    const int gr = std::max(1, std::min(gb, 64));
    if (c.precision == HS_FP64) {
        hipLaunchKernelGGL((k_collide_dense<double, kCapBlockMid, 128>), dim3(2 * gb), dim3(128), 0, S_(s), c, 0, 0);
        hipLaunchKernelGGL((k_collide_dense<double, kCapBlockMax, kBlock>), dim3(gb), dim3(kBlock), 0, S_(s), c, 1, 1);
        hipLaunchKernelGGL((k_collide_dense<double, kCapBlockLds, kBlock>), dim3(gr), dim3(kBlock), 0, S_(s), c, 2, 2);
        hipLaunchKernelGGL((k_collide_dense<double, 1, kBlock, true>), dim3(gr), dim3(kBlock), 0, S_(s), c, 3, 3);
    } else {
        // FP32 classes 0 and 1 in one launch: at 256 threads it already holds two blocks per
        // compute unit, and 128-thread blocks measured slower
        hipLaunchKernelGGL((k_collide_dense<float, kCapBlockMax, kBlock>), dim3(gb), dim3(kBlock), 0, S_(s), c, 0, 1);
        hipLaunchKernelGGL((k_collide_dense<float, kCapBlockLds, kBlock>), dim3(gr), dim3(kBlock), 0, S_(s), c, 2, 2);
        hipLaunchKernelGGL((k_collide_dense<float, 1, kBlock, true>), dim3(gr), dim3(kBlock), 0, S_(s), c, 3, 3);
    }
}
void Launch::finish_step(const Ctx &c, void *s)
{
    hipLaunchKernelGGL(k_finish_step, dim3(1), dim3(256), 0, S_(s), c, c.perm != nullptr ? 1 : 0);
}
void Launch::philox(uint64_t seed, uint32_t stream_id, uint64_t e0, uint32_t step, uint32_t d, int64_t n,
                    uint32_t *out, void *s)
{
    hipLaunchKernelGGL(k_philox, dim3(blocks_for(n, 256)), dim3(256), 0, S_(s), seed, stream_id, e0, step, d, n, out);
}

// Explicit launcher for the current-state moments (needs the case's cell count).
void launch_moments_now(const Ctx &c, void *s, int case_id, int ncells, double *out)
{
    if (c.precision == HS_FP64)
        hipLaunchKernelGGL(k_moments_now<double>, dim3(blocks_for(ncells, 256)), dim3(256), 0, S_(s), c, case_id, out);
    else
        hipLaunchKernelGGL(k_moments_now<float>, dim3(blocks_for(ncells, 256)), dim3(256), 0, S_(s), c, case_id, out);
}

void launch_build_big(const Ctx &c, void *s)
{
    hipLaunchKernelGGL(k_build_big, dim3(blocks_for(c.ncells_total, 256)), dim3(256), 0, S_(s), c);
}

// Wall sums of surface element e of the batch: the kSurfCopies copies added in copy order.
__device__ inline void surf_sums(const Ctx &C, int e, double (&S)[7])
{
    for (int j = 0; j < 7; ++j) S[j] = 0.0;
    for (int c = 0; c < kSurfCopies; ++c) {
        const double *P = C.surf + 7 * ((size_t)c * (size_t)C.n_surf_total + (size_t)e);
        for (int j = 0; j < 7; ++j) S[j] = S[j] + P[j];
    }
}

__global__ void k_surface_reduce(Ctx C, int case_id, double *out)
{
    const CaseDev &cs = C.cases[case_id];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cs.n_surf) return;
    double S[7];
    surf_sums(C, cs.surf0 + k, S);
    for (int j = 0; j < 7; ++j) out[7 * (size_t)k + j] = S[j];
}

void launch_surface_reduce(const Ctx &c, void *s, int case_id, double *out)
{
    const int ns = c.n_surf_total > 0 ? c.n_surf_total : 1;
    hipLaunchKernelGGL(k_surface_reduce, dim3(blocks_for(ns, 256)), dim3(256), 0, S_(s), c, case_id, out);
}

// Time averages of one case's body wall sums: per element the mid angle, area, p, tau, q
// and the Eq. 35 coefficients (with C_f for the shear), then the body force and the Eq. 36
// C_D, C_L (freestream = the case's inflow state).  One block; out holds 8 n_surf + 5.
__global__ void k_surface_finalize(Ctx C, int case_id, double *out)
{
    __shared__ double red[3][256];
    const CaseDev &cs = C.cases[case_id];
    const int ns = cs.n_surf;
    const double R = cs.body_r;
    const double len = cs.dim == 3 ? (double)cs.n[2] * cs.h[2] : cs.h[2];
    const double time = C.g->t_sampled[case_id];
    const double U = sqrt(cs.in_u[0] * cs.in_u[0] + cs.in_u[1] * cs.in_u[1] + cs.in_u[2] * cs.in_u[2]);
    const double rho = cs.in_n * C.gas.m, pinf = cs.in_n * kKB * cs.in_T;
    const double qd = 0.5 * rho * U * U;
    const bool cyl = cs.body == HS_BODY_CYLINDER;
    const double aref = cyl ? 2.0 * R * len : kPi * R * R;
    double F[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < ns; k += blockDim.x) {
        double S[7];
        surf_sums(C, cs.surf0 + k, S);
        const double t0 = kPi * (double)k / (double)ns, t1 = kPi * (double)(k + 1) / (double)ns;
        const double area = cyl ? 2.0 * R * (t1 - t0) * len : 2.0 * kPi * R * R * (cos(t0) - cos(t1));
        double p = 0.0, tau = 0.0, q = 0.0;
        if (time > 0.0) {
            p = -S[1] / (area * time);
            tau = S[2] / (area * time);
            q = S[3] / (area * time);
            for (int a = 0; a < 3; ++a) F[a] = F[a] + S[4 + a] / time;
        }
        double *E = out + 8 * (size_t)k;
        E[0] = 0.5 * (t0 + t1);
        E[1] = area;
        E[2] = p;
        E[3] = tau;
        E[4] = q;
        E[5] = qd > 0.0 ? (p - pinf) / qd : 0.0;
        E[6] = qd > 0.0 ? tau / qd : 0.0;
        E[7] = qd > 0.0 ? q / (qd * U) : 0.0;
    }
    for (int a = 0; a < 3; ++a) red[a][threadIdx.x] = F[a];
    __syncthreads();
    if (threadIdx.x == 0) {
        double Ft[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < (int)blockDim.x; ++j)
            for (int a = 0; a < 3; ++a) Ft[a] = Ft[a] + red[a][j];
        double *B = out + 8 * (size_t)ns;
        double drag = 0.0, lift = 0.0;
        if (U > 0.0) {
            drag = (Ft[0] * cs.in_u[0] + Ft[1] * cs.in_u[1] + Ft[2] * cs.in_u[2]) / U;
            lift = (-Ft[0] * cs.in_u[1] + Ft[1] * cs.in_u[0]) / U;
        }
        for (int a = 0; a < 3; ++a) B[a] = Ft[a];
        B[3] = qd > 0.0 ? drag / (qd * aref) : 0.0;
        B[4] = qd > 0.0 ? lift / (qd * aref) : 0.0;
    }
}

void launch_surface_finalize(const Ctx &c, void *s, int case_id, double *out)
{
    hipLaunchKernelGGL(k_surface_finalize, dim3(1), dim3(256), 0, S_(s), c, case_id, out);
}

// Ratio of DSMC per cell (Eq. 27's Dt_DSMC / Dt_G) from the time-averaged n, U, T of the
// Step (5) sums: 1 where Dt_c <= tau, tau / Dt_c elsewhere (tau of Eq. 10, Dt_c of Eq. 25;
// a 0-D cell's own step); 0 without samples.
__global__ void k_dsmc_ratio(Ctx C, int case_id, double *out)
{
    const CaseDev &cs = C.cases[case_id];
    const int lc = blockIdx.x * blockDim.x + threadIdx.x;
    if (lc >= cs.ncells) return;
    const int g = cs.cell0 + lc;
    const double *A = &C.acc[13 * (size_t)g];
    const double S = (double)C.g->n_samples[case_id];
    const double vol = C.vol[g];
    double r = 0.0;
    if (A[0] > 0.0 && S > 0.0 && vol > 0.0) {
        const double nn = cs.F_N * A[0] / (S * vol);
        double U[3];
        for (int a = 0; a < 3; ++a) U[a] = A[1 + a] / A[0];
        const double cc = (A[4] + A[5] + A[6]) / A[0];
        const double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
        const double T = C.gas.m / (3.0 * kKB) * (cc - uu);
        if (nn > 0.0 && T > 0.0) {
            const double tau = C.gas.mu_ref * pow(T / C.gas.T_ref, C.gas.omega) / (nn * kKB * T);
            const double dtc = cs.dim == 0 ? C.dt_cell[g]
                                           : (cs.mesh ? C.mgeo[2 * (size_t)g + 1] : cs.L_cell) / (sqrt(uu) + sqrt(C.gas.gamma * C.gas.R * T));
            r = dtc <= tau ? 1.0 : tau / dtc;
        }
    }
    out[lc] = r;
}

void launch_dsmc_ratio(const Ctx &c, void *s, int case_id, int ncells, double *out)
{
    hipLaunchKernelGGL(k_dsmc_ratio, dim3(blocks_for(ncells, 256)), dim3(256), 0, S_(s), c, case_id, out);
}

void launch_finalize(const Ctx &c, void *s, int case_id, int ncells, double *out)
{
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(ncells, 256)), dim3(256), 0, S_(s), c, case_id, out);
}

// Fixed scratch array for hs_init_particles_static (sims whose callers cannot allocate device
// memory).  Every device holds its own copy; its address is looked up once per device, with
// that device current, and kept: host code uses only that address, never the array's name.
static __device__ __align__(256) unsigned char scratch[HS_STATIC_SCRATCH_BYTES];

int static_scratch(void **ptr, size_t *bytes)
{
    constexpr int kMaxDevices = 64;
    static std::mutex lock;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(lock);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = (size_t)HS_STATIC_SCRATCH_BYTES;
    return 0;
}

int cap_wave() { return kCapWave; }
int tile_width() { return kTileW; }
int cap_block(int) { return kCapBlockLds; }

}  // namespace hsk
