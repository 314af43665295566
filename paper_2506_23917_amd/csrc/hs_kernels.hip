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

template <typename P>
struct Parts {
    P *pos[3];
    P *vel[3];
    int32_t *cell;
    int64_t *id;
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
        for (int a = 0; a < cs.dim; ++a) {
            const double ctr = cs.lo[a] + ((double)ijk[a] + 0.5) * cs.h[a];
            if (!(ctr >= b[a] && ctr < b[3 + a])) in = false;
        }
        if (in) return &C.region_state[cs.region0 + r];
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
    for (int a = 0; a < cs.dim; ++a) full *= kSub;
    const double vfull = cs.h[0] * cs.h[1] * cs.h[2];
    double vol = vfull;
    if (cs.body != HS_BODY_NONE && cs.dim > 0) vol = (double)cut_count(cs, ijk) / (double)full * vfull;
    C.vol[g] = vol;
    C.sigc[g] = cs.sigc0;
    for (int j = 0; j < 13; ++j) C.acc[13 * (size_t)g + j] = 0.0;
    int N = 0;
    if (fill && vol > 0.0) {
        const StateDev *st = region_of(C, cs, ijk);
        if (st && st->n > 0.0) {
            const W4 w = draw(cs, kStreamInit, (uint64_t)lc, 0, 0);
            N = (int)floor(st->n * vol / cs.F_N + unid(w.x));
        }
    }
    C.count[g] = N;
}

template <typename P>
__global__ void k_init_fill(Ctx C)
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
    const StateDev *st = region_of(C, cs, ijk);
    Parts<P> B(C.buf[0]);
    const int64_t id0 = (int64_t)s - C.cstart[cs.cell0];
    const double a = sqrt(2.0 * C.gas.R * st->T);
    for (int q = 0; q < N; ++q) {
        double xr[3] = {0.0, 0.0, 0.0};
        if (cs.dim > 0) {
            bool placed = false;
            for (int t = 0; t < kMaxPosTry && !placed; ++t) {
                const W4 w = draw(cs, kStreamInit, (uint64_t)lc, 0, (uint32_t)(1 + 128 * q + t));
                const uint32_t ww[3] = {w.x, w.y, w.z};
                double X[3] = {0.0, 0.0, 0.0};
                for (int d = 0; d < cs.dim; ++d) {
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
                            for (int d = 0; d < cs.dim; ++d) {
                                xr[d] = ((double)sub[d] + 0.5) / kSub;
                                X[d] = cs.lo[d] + ((double)ijk[d] + xr[d]) * cs.h[d];
                            }
                            placed = !in_body(cs, X);
                        }
            }
        }
        const W4 w = draw(cs, kStreamInit, (uint64_t)lc, 0, (uint32_t)(1 + 128 * q + 64));
        double s1, c1, s3, c3;
        sincos(2.0 * kPi * unid(w.x), &s1, &c1);
        sincos(2.0 * kPi * unid(w.z), &s3, &c3);
        const double r2 = sqrt(-log(unid(w.y))), r4 = sqrt(-log(unid(w.w)));
        const double C3[3] = {a * c1 * r2, a * c3 * r4, a * s3 * r4};
        const size_t i = (size_t)s + q;
        for (int d = 0; d < 3; ++d) {
            P x = (P)xr[d];
            if (!(x < (P)1)) x = Real<P>::below_one();
            if (d < cs.dim) B.pos[d][i] = x;
            B.vel[d][i] = (P)(st->u[d] + C3[d]);
        }
        B.cell[i] = g;
        B.id[i] = id0 + q;
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
        for (int k = 0; k < HS_NUM_COUNTERS; ++k) G->counters[c][k] = 0;
        if (np > cs.capacity) raise_error(G, kErrCapacity);
    }
    if (t == 0) {
        G->step = step0;
        G->n_live = C.cstart[C.ncells_total];
        G->n_total = G->n_live;
        G->n_new = G->n_live;
        G->n_big = 0;
        G->n_inject = 0;
        if (G->n_live > C.capacity) raise_error(G, kErrCapacity);
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
            if (build_big && v[k] > C.cap_wave) {
                const int slot = atomicAdd(&C.g->n_big, 1);
                C.big_list[slot] = g;
            }
        }
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
    C.face_cnt[f] = (int)floor(fd.lambda + unid(w.x));
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

// One wavefront per inflow face; lanes stride over the face's new particles.
template <typename P>
__global__ void k_inject_fill(Ctx C)
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
        sincos(2.0 * kPi * unid(wv.x), &sn2, &cs2);
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
        S.id[i] = id0 + q;
    }
    if (capped) atomicAdd((unsigned long long *)&C.g->counters[fd.case_id][HS_CNT_INJECT_CAP], (unsigned long long)capped);
}

// ------------------------------------------------------------------------------------
// Free transport and cell counts (Step 2 -> Step 3 histogram)
// ------------------------------------------------------------------------------------

template <typename P>
__device__ __forceinline__ int transport(const Ctx &C, const Parts<P> &S, int i, int g, const CaseDev &cs,
                                         int n_live, uint32_t st, P xr[3], P v[3], int64_t &id, MoveStats &ms)
{
    for (int a = 0; a < cs.dim; ++a) xr[a] = S.pos[a][i];
    for (int a = 0; a < 3; ++a) v[a] = S.vel[a][i];
    if (cs.dim == 0) return g;
    const bool full = i < n_live;
    double t = cs.dt_G;
    if (!full) {
        if (id < 0) id = S.id[i];
        t = cs.dt_G * unid(draw(cs, kStreamParticle, (uint64_t)id, st, kDrawInjectTime).x);
    }
    const int nl = move_particle<P>(C.gas, cs, g - cs.cell0, xr, v, id, &S.id[i], t, full, st, ms);
    return nl >= 0 ? cs.cell0 + nl : -1;
}

template <typename P>
__global__ __launch_bounds__(kBlock) void k_move_count(Ctx C)
{
    Globals *G = C.g;
    if (G->halt) return;
    const int n_total = G->n_total, n_live = G->n_live;
    const uint32_t st = (uint32_t)G->step;
    const Parts<P> S(C.buf[G->step & 1]);
    const int stride = gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    for (int base = blockIdx.x * blockDim.x; base < n_total; base += stride) {
        const int i = base + threadIdx.x;
        const bool valid = i < n_total;
        int nc = -1, cid = 0;
        MoveStats ms{0, 0};
        if (valid) {
            const int g = S.cell[i];
            cid = case_of(C, g);
            const CaseDev &cs = C.cases[cid];
            P xr[3], v[3];
            int64_t id = -1;
            nc = transport<P>(C, S, i, g, cs, n_live, st, xr, v, id, ms);
            C.newcell[i] = nc;
        }
        // wave-aggregated slot allocation in the destination cell
        unsigned long long pending = __ballot(valid && nc >= 0);
        int myslot = 0;
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int c0 = __shfl(nc, leader, 64);
            const unsigned long long same = __ballot(valid && nc == c0) & pending;
            int old = 0;
            if (lane == leader) old = atomicAdd(&C.count[c0], __popcll(same));
            old = __shfl(old, leader, 64);
            if ((same >> lane) & 1ull) myslot = old + __popcll(same & ((1ull << lane) - 1ull));
            pending &= ~same;
        }
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
// Collision stage (Step 3 moments, Step 4, Step 5) for one cell
// ------------------------------------------------------------------------------------

struct CellCounts {
    long long cand, acc, relax, ar, arcap, skipped;
};

// Sort `a[0..p2)` ascending in LDS with a bitonic network (p2 a power of two).
template <int TEAM>
__device__ __forceinline__ void bitonic_sort(int32_t *a, int p2, int tid)
{
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < p2; i += TEAM) {
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
            team_sync<TEAM>();
        }
    }
}

template <typename P, int TEAM>
__device__ void collide_cell(const Ctx &C, int g, int tid, int32_t *s_src, P *s_v, int cap, double *red,
                             long long *redl, int *redi, CellCounts &cc)
{
    Globals *G = C.g;
    const int cid = case_of(C, g);
    const CaseDev &cs = C.cases[cid];
    const GasDev &gas = C.gas;
    const int lc = g - cs.cell0;
    const int64_t step = G->step;
    const uint32_t st = (uint32_t)step;
    const Parts<P> S(C.buf[step & 1]);
    const Parts<P> D(C.buf[(step & 1) ^ 1]);
    const int s = C.cstart[g];
    const int n = C.cstart[g + 1] - s;
    const bool sampling = step >= cs.n_steady;
    const bool tracing = C.trace != nullptr;
    TraceDev tr = {};
    tr.n = n;
    if (n == 0) {
        if (tracing && tid == 0) C.trace[g] = tr;
        return;
    }
    P *vx = s_v, *vy = s_v + cap, *vz = s_v + 2 * cap;

    // sources of this cell in their previous array order
    const bool use_perm = C.perm != nullptr;
    if (use_perm) {
        int p2 = 1;
        while (p2 < n) p2 <<= 1;
        for (int k = tid; k < p2; k += TEAM) s_src[k] = k < n ? C.perm[s + k] : 0x7fffffff;
        team_sync<TEAM>();
        bool unsorted = false;
        for (int k = tid; k + 1 < n; k += TEAM) unsorted |= s_src[k] > s_src[k + 1];
        if (team_any<TEAM>(unsorted, redi)) bitonic_sort<TEAM>(s_src, p2, tid);
    }
    // gather, re-run the move, write position / cell / id of the sorted state
    const int n_live = G->n_live;
    bool bad = false;
    for (int k = tid; k < n; k += TEAM) {
        const int i = use_perm ? s_src[k] : s + k;
        P xr[3], v[3];
        int64_t id = S.id[i];
        MoveStats ms{0, 0};
        if (use_perm) {
            const int nc = transport<P>(C, S, i, S.cell[i], cs, n_live, st, xr, v, id, ms);
            bad |= nc != g;
        } else {
            for (int a = 0; a < cs.dim; ++a) xr[a] = S.pos[a][i];
            for (int a = 0; a < 3; ++a) v[a] = S.vel[a][i];
        }
        const size_t o = (size_t)s + k;
        for (int a = 0; a < cs.dim; ++a) D.pos[a][o] = xr[a];
        D.cell[o] = g;
        D.id[o] = id;
        vx[k] = v[0];
        vy[k] = v[1];
        vz[k] = v[2];
    }
    if (bad) raise_error(G, kErrState);
    team_sync<TEAM>();

    // Eq. 31 moments: mean first, then central sums (FP64 across the team)
    double m1[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = tid; k < n; k += TEAM) {
        const double a = (double)vx[k], b = (double)vy[k], c = (double)vz[k];
        m1[0] = m1[0] + a;
        m1[1] = m1[1] + b;
        m1[2] = m1[2] + c;
        m1[3] = m1[3] + (a * a + b * b + c * c);
    }
    team_sum<TEAM, 4>(m1, red);
    for (int a = 0; a < 4; ++a) tr.pre_sum[a] = m1[a];
    const double U[3] = {m1[0] / (double)n, m1[1] / (double)n, m1[2] / (double)n};
    double m2[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (sizeof(P) == 4) {
        // FP32 peculiar velocities and products with compensated (TwoSum) per-thread sums,
        // FP64 across the team.  C = (c - U_f) - (U - U_f): the first difference is exact
        // for c near U, the second removes the rounding of U to FP32.
        const float uf[3] = {(float)U[0], (float)U[1], (float)U[2]};
        const float df[3] = {(float)(U[0] - (double)uf[0]), (float)(U[1] - (double)uf[1]),
                             (float)(U[2] - (double)uf[2])};
        float sum[4] = {0.f, 0.f, 0.f, 0.f}, cmp[4] = {0.f, 0.f, 0.f, 0.f};
        for (int k = tid; k < n; k += TEAM) {
            const float cx = ((float)vx[k] - uf[0]) - df[0];
            const float cy = ((float)vy[k] - uf[1]) - df[1];
            const float cz = ((float)vz[k] - uf[2]) - df[2];
            const float c2 = cx * cx + cy * cy + cz * cz;
            const float term[4] = {c2, c2 * cx, c2 * cy, c2 * cz};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float t = sum[j] + term[j];
                const float bp = t - sum[j];
                cmp[j] += (sum[j] - (t - bp)) + (term[j] - bp);
                sum[j] = t;
            }
        }
        for (int j = 0; j < 4; ++j) m2[j] = (double)sum[j] + (double)cmp[j];
        team_sum<TEAM, 4>(m2, red);
    } else {
        for (int k = tid; k < n; k += TEAM) {
            const double cx = vx[k] - U[0], cy = vy[k] - U[1], cz = vz[k] - U[2];
            const double c2 = cx * cx + cy * cy + cz * cz;
            m2[0] = m2[0] + c2;
            m2[1] = m2[1] + c2 * cx;
            m2[2] = m2[2] + c2 * cy;
            m2[3] = m2[3] + c2 * cz;
        }
        team_sum<TEAM, 4>(m2, red);
    }
    const double vol = C.vol[g];
    double T = 0.0, Q[3] = {0.0, 0.0, 0.0};
    if (n >= 2) {
        if constexpr (sizeof(P) == 4) {
            // FP32-mixed: T from the FP64 sums sum c and sum |c|^2, the form the FP64
            // rescale restores exactly (energy n|U|^2 + 3k(n-1)T/m)
            const double e = m1[3] - (m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2]) / (double)n;
            T = gas.m * e / (3.0 * kKB * (double)(n - 1));
        } else {
            T = gas.m * m2[0] / (3.0 * kKB * (double)(n - 1));
        }
    }
    if (n >= 3 && vol > 0.0) {
        const double nd = (double)n * cs.F_N / vol;
        const double f = nd * (double)n / ((double)(n - 1) * (double)(n - 2));
        for (int a = 0; a < 3; ++a) Q[a] = f * 0.5 * gas.m * m2[1 + a];
    }
    if (!isfinite(T) || !isfinite(Q[0] + Q[1] + Q[2])) raise_error(G, kErrNumeric);
    const bool active = n >= 2 && T > 0.0 && vol > 0.0;
    if (!active && n >= 2) cc.skipped++;

    if (active) {
        // Eq. 10, 25-28, 16, 5: timescales and sub-step lengths in FP64
        const double nd = (double)n * cs.F_N / vol;
        const double p = nd * kKB * T;
        const double tau = gas.mu_ref * pow(T / gas.T_ref, gas.omega) / p;
        const double dtG = cs.dim == 0 ? C.dt_cell[g] : cs.dt_G;
        double dtc;
        if (cs.dim == 0) {
            dtc = dtG;
        } else {
            const double um = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
            dtc = cs.L_cell / (um + sqrt(gas.gamma * gas.R * T));
        }
        double dtD, dtS;
        if (dtc <= tau) {
            dtD = dtG;
            dtS = 0.0;
        } else {
            dtD = (tau / dtc) * dtG;
            dtS = dtG - dtD;
        }
        const double p_relax = -expm1(-dtS / tau);
        tr.T = T;
        tr.tau = tau;
        tr.dt_dsmc = dtD;
        tr.p_relax = p_relax;
        const double scmax = C.sigc[g];
        const double M = 0.5 * (double)n * (double)(n - 1) * cs.F_N * scmax * dtD / vol;
        const double Mu = M + unid(draw(cs, kStreamCell, (uint64_t)lc, st, 0).x);
        long long ncol = 0;
        if (Mu >= 0.0 && Mu < 1e9) ncol = (long long)floor(Mu);
        else raise_error(G, kErrNumeric);

        // NTC chain (Eq. 5-9), sequential in the candidate index, one thread
        if (tid == 0) {
            const P scm = (P)scmax;
            const P K = (P)gas.K_vhs, ex = (P)gas.vhs_exp;
            double obs = 0.0;
            long long nacc = 0;
            uint64_t hash = 0;
            for (long long k = 0; k < ncol; ++k) {
                const W4 w = draw(cs, kStreamCell, (uint64_t)lc, st, (uint32_t)(1 + 2 * k));
                const uint32_t i = unidx(w.x, (uint32_t)n);
                uint32_t j = unidx(w.y, (uint32_t)(n - 1));
                if (j >= i) ++j;
                const P ua = Real<P>::uni(w.z);
                const P gx = vx[i] - vx[j], gy = vy[i] - vy[j], gz = vz[i] - vz[j];
                const P cr = Real<P>::sq(gx * gx + gy * gy + gz * gz);
                const P sc = K * Real<P>::pw(cr, ex);
                if ((double)sc > obs) obs = (double)sc;
                if (ua < sc / scm) {
                    const W4 w2 = draw(cs, kStreamCell, (uint64_t)lc, st, (uint32_t)(2 + 2 * k));
                    const P cchi = (P)2 * Real<P>::uni(w2.x) - (P)1;
                    const P schi = Real<P>::sq((P)1 - cchi * cchi);
                    P sth, cth;
                    Real<P>::sc((P)(2.0 * kPi) * Real<P>::uni(w2.y), &sth, &cth);
                    const P om[3] = {cchi, schi * cth, schi * sth};
                    P *vv[3] = {vx, vy, vz};
                    for (int a = 0; a < 3; ++a) {
                        const P sum = vv[a][i] + vv[a][j];
                        vv[a][i] = (P)0.5 * (sum - cr * om[a]);
                        vv[a][j] = (P)0.5 * (sum + cr * om[a]);
                    }
                    ++nacc;
                    hash ^= (uint64_t)(k + 1) * 0x9E3779B97F4A7C15ull;
                }
            }
            if (obs > C.sigc[g]) C.sigc[g] = obs;
            tr.ncol = ncol;
            tr.nacc = nacc;
            tr.acc_hash = hash;
            cc.cand += ncol;
            cc.acc += nacc;
        }
        team_sync<TEAM>();

        // SP-Shakhov (Eq. 16-18) from the Step (3) moments
        long long nrel = 0, nar = 0, ncap = 0;
        if (p_relax > 0.0) {
            const double RT = gas.R * T;
            const double qm = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
            const double a_max = 1.0 + 20.0 * (1.0 - gas.Pr) * qm / (p * sqrt(RT));
            tr.a_max = a_max;
            const P am = (P)a_max, one_m_pr = (P)(1.0 - gas.Pr), pP = (P)p, RTP = (P)RT;
            const P ath = (P)sqrt(2.0 * gas.R * T);
            const P QP[3] = {(P)Q[0], (P)Q[1], (P)Q[2]};
            for (int k = tid; k < n; k += TEAM) {
                const int64_t id = D.id[(size_t)s + k];
                if (!(unid(draw(cs, kStreamParticle, (uint64_t)id, st, kDrawRelax).x) < p_relax)) continue;
                ++nrel;
                P Cv[3];
                int used = -kMaxShakhov;
                for (int a = 0; a < kMaxShakhov; ++a) {
                    const W4 w = draw(cs, kStreamParticle, (uint64_t)id, st, kDrawShakhov + 2 * a);
                    const W4 w5 = draw(cs, kStreamParticle, (uint64_t)id, st, kDrawShakhov + 2 * a + 1);
                    P s1, c1, s3, c3;
                    Real<P>::sc((P)(2.0 * kPi) * Real<P>::uni(w.x), &s1, &c1);
                    Real<P>::sc((P)(2.0 * kPi) * Real<P>::uni(w.z), &s3, &c3);
                    const P r2 = Real<P>::sq(-Real<P>::ln(Real<P>::uni(w.y)));
                    const P r4 = Real<P>::sq(-Real<P>::ln(Real<P>::uni(w.w)));
                    Cv[0] = ath * c1 * r2;
                    Cv[1] = ath * c3 * r4;
                    Cv[2] = ath * s3 * r4;
                    const P c2 = Cv[0] * Cv[0] + Cv[1] * Cv[1] + Cv[2] * Cv[2];
                    const P qc = QP[0] * Cv[0] + QP[1] * Cv[1] + QP[2] * Cv[2];
                    const P A = (P)1 + one_m_pr * qc / ((P)5 * pP * RTP) * (c2 / RTP - (P)5);
                    if (A / am > Real<P>::uni(w5.x)) {
                        used = a + 1;
                        break;
                    }
                }
                if (used < 0) {
                    ++ncap;
                    used = -used;
                }
                nar += used;
                vx[k] = (P)(U[0] + (double)Cv[0]);
                vy[k] = (P)(U[1] + (double)Cv[1]);
                vz[k] = (P)(U[2] + (double)Cv[2]);
            }
        }
        long long sl[3] = {nrel, nar, ncap};
        team_sum_i<TEAM, 3>(sl, redl);
        tr.nrelax = sl[0];
        tr.ar_attempts = sl[1];
        tr.ar_cap = sl[2];
        if (tid == 0) {
            cc.relax += sl[0];
            cc.ar += sl[1];
            cc.arcap += sl[2];
        }
        team_sync<TEAM>();

        // Eq. 19 conservation rescale in FP64 with the Step (3) U and T
        double r1[3] = {0.0, 0.0, 0.0};
        for (int k = tid; k < n; k += TEAM) {
            r1[0] = r1[0] + (double)vx[k];
            r1[1] = r1[1] + (double)vy[k];
            r1[2] = r1[2] + (double)vz[k];
        }
        team_sum<TEAM, 3>(r1, red);
        const double Up[3] = {r1[0] / (double)n, r1[1] / (double)n, r1[2] / (double)n};
        double r2[1] = {0.0};
        for (int k = tid; k < n; k += TEAM) {
            const double cx = (double)vx[k] - Up[0], cy = (double)vy[k] - Up[1], cz = (double)vz[k] - Up[2];
            r2[0] = r2[0] + (cx * cx + cy * cy + cz * cz);
        }
        team_sum<TEAM, 1>(r2, red);
        const double Tp = gas.m * r2[0] / (3.0 * kKB * (double)(n - 1));
        double post[4] = {0.0, 0.0, 0.0, 0.0};
        if (Tp > 0.0) {
            const double f = sqrt(T / Tp);
            for (int k = tid; k < n; k += TEAM) {
                const double a = U[0] + ((double)vx[k] - Up[0]) * f;
                const double b = U[1] + ((double)vy[k] - Up[1]) * f;
                const double c = U[2] + ((double)vz[k] - Up[2]) * f;
                post[0] = post[0] + a;
                post[1] = post[1] + b;
                post[2] = post[2] + c;
                post[3] = post[3] + (a * a + b * b + c * c);
                vx[k] = (P)a;
                vy[k] = (P)b;
                vz[k] = (P)c;
            }
        }
        if (tracing) {
            if (Tp > 0.0) {
                team_sum<TEAM, 4>(post, red);
                for (int a = 0; a < 4; ++a) tr.post_sum[a] = post[a];
            } else {
                for (int a = 0; a < 4; ++a) tr.post_sum[a] = 0.0;
            }
        }
        team_sync<TEAM>();
    }

    // write velocities; Step (5) sums of the final state
    double sm[12];
    for (int j = 0; j < 12; ++j) sm[j] = 0.0;
    for (int k = tid; k < n; k += TEAM) {
        const size_t o = (size_t)s + k;
        const P a = vx[k], b = vy[k], c = vz[k];
        D.vel[0][o] = a;
        D.vel[1][o] = b;
        D.vel[2][o] = c;
        if (sampling || (tracing && !active)) {
            const double x = (double)a, y = (double)b, z = (double)c;
            const double c2 = x * x + y * y + z * z;
            sm[0] = sm[0] + x;
            sm[1] = sm[1] + y;
            sm[2] = sm[2] + z;
            sm[3] = sm[3] + x * x;
            sm[4] = sm[4] + y * y;
            sm[5] = sm[5] + z * z;
            sm[6] = sm[6] + x * y;
            sm[7] = sm[7] + x * z;
            sm[8] = sm[8] + y * z;
            sm[9] = sm[9] + c2 * x;
            sm[10] = sm[10] + c2 * y;
            sm[11] = sm[11] + c2 * z;
        }
    }
    if (sampling || (tracing && !active)) team_sum<TEAM, 12>(sm, red);
    if (tracing && !active) {
        tr.post_sum[0] = sm[0];
        tr.post_sum[1] = sm[1];
        tr.post_sum[2] = sm[2];
        tr.post_sum[3] = sm[3] + sm[4] + sm[5];
    }
    if (tid == 0) {
        if (sampling) {
            double *A = &C.acc[13 * (size_t)g];
            A[0] += (double)n;
            for (int j = 0; j < 12; ++j) A[1 + j] += sm[j];
        }
        if (tracing) C.trace[g] = tr;
    }
    team_sync<TEAM>();
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

// One wavefront per cell of at most CAPW particles; four wavefronts per block.
template <typename P, int CAPW>
__global__ __launch_bounds__(kBlock) void k_collide_wave(Ctx C)
{
    if (C.g->halt) return;
    __shared__ int32_t s_src[4][CAPW];
    __shared__ P s_v[4][3 * CAPW];
    __shared__ double red[4][16];
    __shared__ long long redl[4][8];
    __shared__ int redi[4][2];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * 4;
    CellCounts cc{0, 0, 0, 0, 0, 0};
    int cur_case = -1;
    for (int g = blockIdx.x * 4 + w; g < C.ncells_total; g += nwaves) {
        const int n = C.cstart[g + 1] - C.cstart[g];
        if (n > CAPW) continue;
        const int cid = case_of(C, g);
        if (cid != cur_case) {
            if (cur_case >= 0 && lane == 0) flush_counts(C, cur_case, cc);
            cur_case = cid;
        }
        collide_cell<P, 64>(C, g, lane, s_src[w], s_v[w], CAPW, red[w], redl[w], redi[w], cc);
    }
    if (cur_case >= 0 && lane == 0) flush_counts(C, cur_case, cc);
}

// One 256-thread block per dense cell (more than the wave kernel's limit).
template <typename P, int CAPB>
__global__ __launch_bounds__(kBlock) void k_collide_block(Ctx C)
{
    if (C.g->halt) return;
    __shared__ int32_t s_src[CAPB];
    __shared__ P s_v[3 * CAPB];
    __shared__ double red[4 * 16];
    __shared__ long long redl[4 * 8];
    __shared__ int redi[2];
    const int nbig = C.g->n_big;
    CellCounts cc{0, 0, 0, 0, 0, 0};
    for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
        const int g = C.big_list[b];
        const int n = C.cstart[g + 1] - C.cstart[g];
        if (n > CAPB) {
            if (threadIdx.x == 0) raise_error(C.g, kErrCellLimit);
            continue;
        }
        collide_cell<P, kBlock>(C, g, threadIdx.x, s_src, s_v, CAPB, red, redl, redi, cc);
        if (threadIdx.x == 0) flush_counts(C, case_of(C, g), cc);
    }
}

// Dense-cell list of a batch whose cells never re-sort (only 0-D cases): built once.
__global__ void k_build_big(Ctx C)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= C.ncells_total) return;
    if (C.cstart[g + 1] - C.cstart[g] > C.cap_wave) {
        const int slot = atomicAdd(&C.g->n_big, 1);
        C.big_list[slot] = g;
    }
}

__global__ void k_finish_step(Ctx C, int sorted)
{
    Globals *G = C.g;
    if (G->halt) return;
    const int64_t step = G->step;
    for (int c = threadIdx.x; c < C.n_cases; c += blockDim.x)
        if (step >= C.cases[c].n_steady) G->n_samples[c] += 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (sorted) {
            G->n_live = G->n_new;
            G->n_big = 0;      // rebuilt by the next step's scan
        }
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

constexpr int kCapWave = 256;
constexpr int kCapBlock64 = 2048;   // powers of two: the bitonic sort pads to one
constexpr int kCapBlock32 = 2048;

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
void Launch::scan_cells(const Ctx &c, void *s, int build_big)
{
    const int nparts = blocks_for(c.ncells_total, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nparts), dim3(kBlock), 0, S_(s), c);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, S_(s), c, nparts);
    hipLaunchKernelGGL(k_scan_final, dim3(nparts), dim3(kBlock), 0, S_(s), c, build_big, nparts);
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
void Launch::move_count(const Ctx &c, void *s)
{
    const int grid = std::min(stream_grid(), blocks_for(c.capacity, kBlock));
    if (c.precision == HS_FP64)
        hipLaunchKernelGGL(k_move_count<double>, dim3(grid), dim3(kBlock), 0, S_(s), c);
    else
        hipLaunchKernelGGL(k_move_count<float>, dim3(grid), dim3(kBlock), 0, S_(s), c);
}
void Launch::scatter(const Ctx &c, void *s)
{
    const int grid = std::min(stream_grid(), blocks_for(c.capacity, kBlock));
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(kBlock), 0, S_(s), c);
}
void Launch::collide(const Ctx &c, void *s)
{
    const int gw = std::max(1, std::min(blocks_for(c.ncells_total, 4), 256 * 8));
    const int gb = std::max(1, std::min(c.ncells_total, 256 * 2));
    if (c.precision == HS_FP64) {
        hipLaunchKernelGGL((k_collide_wave<double, kCapWave>), dim3(gw), dim3(kBlock), 0, S_(s), c);
        hipLaunchKernelGGL((k_collide_block<double, kCapBlock64>), dim3(gb), dim3(kBlock), 0, S_(s), c);
    } else {
        hipLaunchKernelGGL((k_collide_wave<float, kCapWave>), dim3(gw), dim3(kBlock), 0, S_(s), c);
        hipLaunchKernelGGL((k_collide_block<float, kCapBlock32>), dim3(gb), dim3(kBlock), 0, S_(s), c);
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

void launch_finalize(const Ctx &c, void *s, int case_id, int ncells, double *out)
{
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(ncells, 256)), dim3(256), 0, S_(s), c, case_id, out);
}

int cap_wave() { return kCapWave; }
int cap_block(int precision) { return precision == HS_FP64 ? kCapBlock64 : kCapBlock32; }

}  // namespace hsk
