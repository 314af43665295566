// hs_device.hpp -- device building blocks of the gfx950 particle update: the counter-based
// generator, uniform conversions, the VHS gas model, Maxwellian draws, the body geometry
// and the free-flight move shared by the move/count and collide kernels (the collide kernel
// re-runs the move of each particle it gathers, bit-identically, instead of storing it).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hs_common.hpp"

namespace hsk {

// Where a particle's id is loaded from when first needed: its stored low 32 bits and the
// case's next id (full_id).
struct IdSrc {
    const uint32_t *low;
    int64_t next;
    __device__ int64_t get() const { return full_id(*low, next); }
};

constexpr double kKB = 1.380649e-23;
constexpr double kPi = 3.14159265358979323846;

struct W4 {
    uint32_t x, y, z, w;
};

// Philox4x32 with ten rounds (Salmon et al., SC'11): per round the first and third
// counter words are multiplied by the two round constants; the high halves are xored
// with the other words and the key; the key advances by the two Weyl increments.
__device__ __forceinline__ W4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product per multiplier (a single v_mad_u64_u32) gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
        const uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
        const uint32_t n0 = h1 ^ c1 ^ k0;
        const uint32_t n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return W4{c0, c1, c2, c3};
}

// Counter = (entity low word, entity bits 32..59 | stream << 28, step, draw); key = seed.
__device__ __forceinline__ W4 draw(const CaseDev &cs, uint32_t stream, uint64_t entity,
                                   uint32_t step, uint32_t d)
{
    return philox10((uint32_t)entity, ((uint32_t)(entity >> 32) & 0x0fffffffu) | (stream << 28),
                    step, d, cs.seed_lo, cs.seed_hi);
}

// The same draw with the case's seed words passed directly.
__device__ __forceinline__ W4 draw_s(uint32_t seed_lo, uint32_t seed_hi, uint32_t stream, uint64_t entity,
                                     uint32_t step, uint32_t d)
{
    return philox10((uint32_t)entity, ((uint32_t)(entity >> 32) & 0x0fffffffu) | (stream << 28), step, d,
                    seed_lo, seed_hi);
}

// 32-bit word -> double uniform in (0,1): (w + 1/2) 2^-32.
__device__ __forceinline__ double unid(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }
// 32-bit word -> float uniform in (0,1): an odd multiple of 2^-24, exactly representable.
__device__ __forceinline__ float unif(uint32_t w) { return (float)(((w >> 9) << 1) | 1u) * 0x1p-24f; }
// 32-bit word -> integer in [0, n): floor(w n / 2^32).
__device__ __forceinline__ uint32_t unidx(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

template <typename P> struct Real;
template <> struct Real<double> {
    __device__ static double uni(uint32_t w) { return unid(w); }
    __device__ static double sq(double x) { return sqrt(x); }
    __device__ static double ln(double x) { return log(x); }
    __device__ static double pw(double x, double y) { return pow(x, y); }
    // sin and cos of 2 pi u for u in (0,1), without a large-argument reduction
    __device__ static void sc2pi(double u, double *s, double *c) { sincospi(2.0 * u, s, c); }
    __device__ static double fl(double x) { return floor(x); }
    __device__ static double below_one() { return 0x1.fffffffffffffp-1; }
};
// FP32 sampling arithmetic on the hardware transcendental units (a few ulp): square root,
// log2 (scaled to ln) and the sine / cosine of a turn fraction (v_sin / v_cos take their
// argument in turns, so 2 pi u needs no range reduction for u in (0, 1)).
template <> struct Real<float> {
    __device__ static float uni(uint32_t w) { return unif(w); }
    __device__ static float sq(float x) { return __builtin_amdgcn_sqrtf(x); }
    __device__ static float ln(float x) { return __builtin_amdgcn_logf(x) * 0x1.62e430p-1f; }
    __device__ static float pw(float x, float y) { return powf(x, y); }
    __device__ static void sc2pi(float u, float *s, float *c)
    {
        *s = __builtin_amdgcn_sinf(u);
        *c = __builtin_amdgcn_cosf(u);
    }
    __device__ static float fl(float x) { return floorf(x); }
    __device__ static float below_one() { return 0x1.fffffep-1f; }
};

// Case of a global cell: binary search over the cases' first cells.
// Reads through the constant address space, for tables that no kernel writes while another
// reads them (the case table; the tile table, written by an earlier launch): wave-uniform
// reads then become scalar loads.
template <typename T>
__device__ __forceinline__ T const_read(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)p;
}

__device__ __forceinline__ const CaseDev &case_const(const Ctx &C, int ci)
{
    using ConstCase = const __attribute__((address_space(4))) CaseDev;
    return *(const CaseDev *)((ConstCase *)C.cases + ci);
}

__device__ __forceinline__ int case_of(const Ctx &C, int g)
{
    int lo = 0, hi = C.n_cases - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (case_const(C, mid).cell0 <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void cell_ijk(const CaseDev &cs, int local, int ijk[3])
{
    ijk[0] = ijk[1] = ijk[2] = 0;
    if (cs.dim == 0) { ijk[0] = local; return; }
    ijk[0] = local % cs.n[0];
    if (cs.dim >= 2) ijk[1] = (local / cs.n[0]) % cs.n[1];
    if (cs.dim >= 3) ijk[2] = local / (cs.n[0] * cs.n[1]);
}

// a / n for 0 <= a < 2^31, n >= 1, from a double reciprocal (a few instructions instead of an
// integer division), corrected to the exact quotient; r = a - q n.
__device__ __forceinline__ int div_exact(int a, int n, double inv, int &r)
{
    int q = (int)((double)a * inv);
    r = a - q * n;
    if (r < 0) {
        --q;
        r += n;
    } else if (r >= n) {
        ++q;
        r -= n;
    }
    return q;
}

// cell_ijk for a grid case (dim 1-3) by reciprocal multiplication.
__device__ __forceinline__ void cell_ijk_fast(const CaseDev &cs, int local, int ijk[3])
{
    ijk[0] = local;
    ijk[1] = ijk[2] = 0;
    if (cs.dim == 3) {
        int rem;
        ijk[2] = div_exact(local, cs.n[0] * cs.n[1], cs.inv_n[1], rem);
        ijk[1] = div_exact(rem, cs.n[0], cs.inv_n[0], ijk[0]);
    } else if (cs.dim == 2) {
        ijk[1] = div_exact(local, cs.n[0], cs.inv_n[0], ijk[0]);
    }
}

__device__ __forceinline__ int cell_local(const CaseDev &cs, const int ijk[3])
{
    return ijk[0] + cs.n[0] * (ijk[1] + cs.n[1] * ijk[2]);
}

__device__ __forceinline__ int body_axes(const CaseDev &cs) { return cs.body == HS_BODY_SPHERE ? 3 : 2; }

// Strictly inside the body: |x - c|^2 < R^2 summed over the body's axes in order x, y, z.
__device__ __forceinline__ bool in_body(const CaseDev &cs, const double X[3])
{
    if (cs.body == HS_BODY_NONE) return false;
    const int na = body_axes(cs);
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) if (a < na) {
        const double d = X[a] - cs.body_c[a];
        d2 = d2 + d * d;
    }
    return d2 < cs.body_r * cs.body_r;
}

// Cut-cell rule: number of the 16^dim sub-cell centres lo + (i + (s + 1/2)/16) h outside
// the body; cells clearly outside / inside (1e-9 relative margin) are classified without
// sampling.
__device__ inline int cut_count(const CaseDev &cs, const int ijk[3])
{
    int full = 1;
    for (int a = 0; a < 3; ++a) if (a < cs.dim) full *= kSub;
    if (cs.body == HS_BODY_NONE || cs.dim == 0) return full;
    const int na = body_axes(cs);
    double near2 = 0.0, far2 = 0.0;
    for (int a = 0; a < 3; ++a) if (a < na) {
        const double blo = cs.lo[a] + (double)ijk[a] * cs.h[a];
        const double bhi = cs.lo[a] + (double)(ijk[a] + 1) * cs.h[a];
        double dn = 0.0;
        if (cs.body_c[a] < blo) dn = blo - cs.body_c[a];
        else if (cs.body_c[a] > bhi) dn = cs.body_c[a] - bhi;
        const double d1 = fabs(blo - cs.body_c[a]), d2 = fabs(bhi - cs.body_c[a]);
        const double df = d2 > d1 ? d2 : d1;
        near2 = near2 + dn * dn;
        far2 = far2 + df * df;
    }
    const double R2 = cs.body_r * cs.body_r;
    if (near2 > R2 * (1.0 + 1e-9)) return full;
    if (far2 < R2 * (1.0 - 1e-9)) return 0;
    int out = 0;
    const int s2n = cs.dim >= 3 ? kSub : 1, s1n = cs.dim >= 2 ? kSub : 1;
    for (int s2 = 0; s2 < s2n; ++s2)
        for (int s1 = 0; s1 < s1n; ++s1)
            for (int s0 = 0; s0 < kSub; ++s0) {
                const int sub[3] = {s0, s1, s2};
                double X[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < cs.dim; ++a)
                    X[a] = cs.lo[a] + ((double)ijk[a] + ((double)sub[a] + 0.5) / kSub) * cs.h[a];
                if (!in_body(cs, X)) ++out;
            }
    return out;
}

// First time the path X + V t meets the body surface within [0, t], or -1.
__device__ __forceinline__ double body_hit(const CaseDev &cs, const double X[3], const double V[3], double t)
{
    const int na = body_axes(cs);
    double a = 0.0, b = 0.0, q = 0.0;
    for (int k = 0; k < 3; ++k) if (k < na) {
        const double d = X[k] - cs.body_c[k];
        a = a + V[k] * V[k];
        b = b + d * V[k];
        q = q + d * d;
    }
    q = q - cs.body_r * cs.body_r;
    if (!(a > 0.0) || q < 0.0 || b >= 0.0) return -1.0;
    const double disc = b * b - a * q;
    if (disc < 0.0) return -1.0;
    const double th = q / (-b + sqrt(disc));
    return th <= t ? th : -1.0;
}

// Diffuse re-emission at the body (full accommodation at body_T): normal speed
// sqrt(2RT_w) sqrt(-ln R1), tangential speeds sqrt(2RT_w) {cos, sin}(2 pi R3) sqrt(-ln R4)
// along t1 and t2 (cylinder: t1 = (-n_y, n_x, 0), t2 = z; sphere: t1 = e x n normalised,
// e the axis of smallest |n_e|, t2 = n x t1).
// Outward unit normal of the body at the wall point X.
__device__ __forceinline__ void body_normal(const CaseDev &cs, const double X[3], double nr[3])
{
    const int na = body_axes(cs);
    double len = 0.0;
    for (int k = 0; k < 3; ++k) nr[k] = 0.0;
    for (int k = 0; k < 3; ++k) if (k < na) {
        nr[k] = X[k] - cs.body_c[k];
        len = len + nr[k] * nr[k];
    }
    len = sqrt(len);
    for (int k = 0; k < 3; ++k) if (k < na) nr[k] = nr[k] / len;
}

// The re-emission about a given unit wall normal nr (pointing into the gas); a mesh wall
// uses the planar frame of the cylinder.
__device__ inline void diffuse_reflect_n(const GasDev &gas, const CaseDev &cs, const double nr[3], W4 w,
                                         double V[3])
{
    double t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
    if ((cs.mesh && cs.dim == 2) || cs.body == HS_BODY_CYLINDER) {
        t1[0] = -nr[1];
        t1[1] = nr[0];
        t2[2] = 1.0;
    } else {
        int e = 0;
        if (fabs(nr[1]) < fabs(nr[e])) e = 1;
        if (fabs(nr[2]) < fabs(nr[e])) e = 2;
        double ev[3] = {0.0, 0.0, 0.0};
        ev[e] = 1.0;
        t1[0] = ev[1] * nr[2] - ev[2] * nr[1];
        t1[1] = ev[2] * nr[0] - ev[0] * nr[2];
        t1[2] = ev[0] * nr[1] - ev[1] * nr[0];
        const double l1 = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
        for (int k = 0; k < 3; ++k) t1[k] = t1[k] / l1;
        t2[0] = nr[1] * t1[2] - nr[2] * t1[1];
        t2[1] = nr[2] * t1[0] - nr[0] * t1[2];
        t2[2] = nr[0] * t1[1] - nr[1] * t1[0];
    }
    const double a = sqrt(2.0 * gas.R * cs.body_T);
    const double cn = a * sqrt(-log(unid(w.x)));
    const double rr = sqrt(-log(unid(w.z)));
    double sn, cs_;
    sincospi(2.0 * unid(w.y), &sn, &cs_);
    const double ct1 = a * cs_ * rr, ct2 = a * sn * rr;
    for (int k = 0; k < 3; ++k) V[k] = cn * nr[k] + ct1 * t1[k] + ct2 * t2[k];
}

__device__ inline void diffuse_reflect(const GasDev &gas, const CaseDev &cs, const double X[3], W4 w,
                                       double V[3])
{
    double nr[3];
    body_normal(cs, X, nr);
    diffuse_reflect_n(gas, cs, nr, w, V);
}

struct MoveStats {
    int hits, capped;
};

// Free flight (Eq. 4) for time t of one particle stored as (cell, cell-relative position
// xr in [0,1)^dim, velocity v): body reflections in FP64 on absolute coordinates, plain
// flight in cell units in the storage precision, specular walls by mirroring, removal
// through open faces.  Returns the new case-local cell or -1.
// `id` is the particle id, or -1 to load it from idsrc on the first body reflection.
// Step (5) on the wall: the momentum dP = m F_N (c_in - c_out) and the energy
// dE = m F_N (|c_in|^2 - |c_out|^2) / 2 one diffuse reflection gives the body, added to the
// surface element of the hit point X.  Elements are bands of the polar angle th from the
// upstream stagnation direction -x; dP is split on the outward normal n and on the unit
// tangent of growing th, t = (n cos th + x) / sin th (zero at the poles).
// (On a mesh wall, n is the unit normal of the edge hit.)
__device__ inline void surface_hit_n(const GasDev &gas, const CaseDev &cs, const double nr[3], const double Vin[3],
                                     const double Vout[3], double *surf)
{
    double ct = -nr[0];
    ct = ct > 1.0 ? 1.0 : (ct < -1.0 ? -1.0 : ct);
    const double th = acos(ct);
    const double st = sin(th);
    const double sdir[3] = {-1.0, 0.0, 0.0};
    double tg[3];
    for (int k = 0; k < 3; ++k) tg[k] = st > 0.0 ? (nr[k] * ct - sdir[k]) / st : 0.0;
    int e = (int)floor(th / kPi * (double)cs.n_surf);
    e = e < 0 ? 0 : (e > cs.n_surf - 1 ? cs.n_surf - 1 : e);
    const double w = gas.m * cs.F_N;
    double dP[3], ein = 0.0, eout = 0.0;
    for (int a = 0; a < 3; ++a) {
        dP[a] = w * (Vin[a] - Vout[a]);
        ein = ein + Vin[a] * Vin[a];
        eout = eout + Vout[a] * Vout[a];
    }
    double *S = surf + 7 * (size_t)(cs.surf0 + e);
    unsafeAtomicAdd(&S[0], 1.0);
    unsafeAtomicAdd(&S[1], dP[0] * nr[0] + dP[1] * nr[1] + dP[2] * nr[2]);
    unsafeAtomicAdd(&S[2], dP[0] * tg[0] + dP[1] * tg[1] + dP[2] * tg[2]);
    unsafeAtomicAdd(&S[3], 0.5 * w * (ein - eout));
    for (int a = 0; a < 3; ++a) unsafeAtomicAdd(&S[4 + a], dP[a]);
}

__device__ inline void surface_hit(const GasDev &gas, const CaseDev &cs, const double X[3], const double Vin[3],
                                   const double Vout[3], double *surf)
{
    double nr[3];
    body_normal(cs, X, nr);
    surface_hit_n(gas, cs, nr, Vin, Vout, surf);
}

template <typename P>
__device__ inline int move_particle(const GasDev &gas, const CaseDev &cs, int local, P xr[3], P v[3],
                                    int64_t &id, IdSrc idsrc, double t, bool full_step,
                                    uint32_t step, MoveStats &ms, double *surf)
{
    const int dim = cs.dim;
    int ijk[3];
    cell_ijk_fast(cs, local, ijk);
    if (cs.body != HS_BODY_NONE) {
        double X[3] = {0.0, 0.0, 0.0}, V[3];
        for (int a = 0; a < 3; ++a) if (a < dim) X[a] = cs.lo[a] + ((double)ijk[a] + (double)xr[a]) * cs.h[a];
        for (int a = 0; a < 3; ++a) V[a] = (double)v[a];
        bool bounced = false;
        for (int b = 0;; ++b) {
            const double th = body_hit(cs, X, V, t);
            if (th < 0.0) break;
            for (int a = 0; a < 3; ++a) if (a < dim) X[a] = X[a] + V[a] * th;
            t = t - th;
            ms.hits++;
            bounced = true;
            if (b == kMaxBounce) {
                ms.capped++;
                t = 0.0;
                break;
            }
            if (id < 0) id = idsrc.get();
            const double Vin[3] = {V[0], V[1], V[2]};
            diffuse_reflect(gas, cs, X, draw(cs, kStreamParticle, (uint64_t)id, step, kDrawBounce + b), V);
            if (surf) surface_hit(gas, cs, X, Vin, V, surf);
        }
        if (bounced) {
            for (int a = 0; a < 3; ++a) if (a < dim) {
                X[a] = X[a] + V[a] * t;
                const double hi = cs.lo[a] + (double)cs.n[a] * cs.h[a];
                if (X[a] < cs.lo[a]) {
                    if (cs.bc[2 * a] != HS_BC_SPECULAR) return -1;
                    X[a] = 2.0 * cs.lo[a] - X[a];
                    V[a] = -V[a];
                } else if (X[a] >= hi) {
                    if (cs.bc[2 * a + 1] != HS_BC_SPECULAR) return -1;
                    X[a] = 2.0 * hi - X[a];
                    V[a] = -V[a];
                }
                const double f = (X[a] - cs.lo[a]) / cs.h[a];
                int i = (int)floor(f);
                i = i < 0 ? 0 : (i > cs.n[a] - 1 ? cs.n[a] - 1 : i);
                double r = f - (double)i;
                P rp = (P)r;
                if (!(rp >= (P)0)) rp = (P)0;
                if (!(rp < (P)1)) rp = Real<P>::below_one();
                xr[a] = rp;
                ijk[a] = i;
            }
            for (int a = 0; a < 3; ++a) v[a] = (P)V[a];
            return cell_local(cs, ijk);
        }
    }
    for (int a = 0; a < 3; ++a) if (a < dim) {
        const P dth = (full_step && !cs.adapt_dt) ? (P)cs.dt_over_h[a] : (P)(t / cs.h[a]);
        P x = xr[a] + v[a] * dth;
        const P f = Real<P>::fl(x);
        int i = ijk[a] + (int)f;
        x = x - f;
        if (x >= (P)1) { x = x - (P)1; i += 1; }
        const int n = cs.n[a];
        if (i < 0) {
            if (cs.bc[2 * a] != HS_BC_SPECULAR) return -1;
            i = -i - 1;
            x = (P)1 - x;
            v[a] = -v[a];
        } else if (i >= n) {
            if (cs.bc[2 * a + 1] != HS_BC_SPECULAR) return -1;
            i = 2 * n - 1 - i;
            x = (P)1 - x;
            v[a] = -v[a];
        }
        if (x >= (P)1) { x = x - (P)1; i += 1; }
        if (i < 0) { i = 0; ms.capped++; }
        if (i > n - 1) { i = n - 1; ms.capped++; }
        xr[a] = x;
        ijk[a] = i;
    }
    return cell_local(cs, ijk);
}

// Whether the flight x + c s, 0 <= s <= t, from the particle's absolute position (formed as
// the body-reflection path forms it, in FP64) comes within the body radius (1 + 1e-9) of the
// body's centre: a conservative test, so every path that the exact FP64 intersection of
// k_move_body would find hitting the wall is sent there, and the others fly here.
template <typename P>
__device__ __forceinline__ bool may_hit_body(const CaseDev &cs, const int ijk[3], const P xr[3], const P v[3],
                                             double t)
{
    const int na = body_axes(cs);
    double d[3] = {0.0, 0.0, 0.0}, w[3] = {0.0, 0.0, 0.0};
    double dv = 0.0, vv = 0.0;
    for (int k = 0; k < 3; ++k) if (k < na) {
        d[k] = cs.lo[k] + ((double)ijk[k] + (double)xr[k]) * cs.h[k] - cs.body_c[k];
        w[k] = (double)v[k];
        dv = dv + d[k] * w[k];
        vv = vv + w[k] * w[k];
    }
    double sm = vv > 0.0 ? -dv / vv : 0.0;
    sm = sm < 0.0 ? 0.0 : (sm > t ? t : sm);
    double m2 = 0.0;
    for (int k = 0; k < 3; ++k) if (k < na) {
        const double e = d[k] + w[k] * sm;
        m2 = m2 + e * e;
    }
    const double r = cs.body_r * (1.0 + 1e-9);
    return m2 <= r * r;
}

// Plain flight (Eq. 4) in cell units for particles that cannot meet the body this step:
// specular walls by mirroring, removal through open faces.  Returns the new case-local
// cell, -1 when the particle left, or -2 when the straight path may meet the body (its
// cell box overlaps the body's and may_hit_body holds; the caller then runs move_particle
// on the untouched state).  vchg is set when a wall changed the velocity.
template <typename P>
__device__ __forceinline__ int flight(const CaseDev &cs, int local, P xr[3], P v[3], double t, bool full_step,
                                      bool &vchg)
{
    const int dim = cs.dim;
    int ijk[3];
    cell_ijk_fast(cs, local, ijk);
    if (cs.body != HS_BODY_NONE) {
        const int na = body_axes(cs);
        bool near = true;
        for (int a = 0; a < 3; ++a) if (a < na) {
            const P dth = (full_step && !cs.adapt_dt) ? (P)cs.dt_over_h[a] : (P)(t / cs.h[a]);
            const P x = xr[a] + v[a] * dth;
            const int i = ijk[a] + (int)Real<P>::fl(x);
            const int lo = i < ijk[a] ? i : ijk[a], hi = i < ijk[a] ? ijk[a] : i;
            if (hi < cs.bb_lo[a] || lo > cs.bb_hi[a]) near = false;
        }
        if (near && may_hit_body(cs, ijk, xr, v, t)) return -2;
    }
    vchg = false;
    for (int a = 0; a < 3; ++a) if (a < dim) {
        const P dth = (full_step && !cs.adapt_dt) ? (P)cs.dt_over_h[a] : (P)(t / cs.h[a]);
        P x = xr[a] + v[a] * dth;
        const P f = Real<P>::fl(x);
        int i = ijk[a] + (int)f;
        x = x - f;
        if (x >= (P)1) { x = x - (P)1; i += 1; }
        const int n = cs.n[a];
        if (i < 0) {
            if (cs.bc[2 * a] != HS_BC_SPECULAR) return -1;
            i = -i - 1;
            x = (P)1 - x;
            v[a] = -v[a];
            vchg = true;
        } else if (i >= n) {
            if (cs.bc[2 * a + 1] != HS_BC_SPECULAR) return -1;
            i = 2 * n - 1 - i;
            x = (P)1 - x;
            v[a] = -v[a];
            vchg = true;
        }
        if (x >= (P)1) { x = x - (P)1; i += 1; }
        i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
        xr[a] = x;
        ijk[a] = i;
    }
    return cell_local(cs, ijk);
}

// ------------------------------------------------------------------------------------
// Quad meshes
// ------------------------------------------------------------------------------------

// The four nodes of global mesh cell g (counter-clockwise).
__device__ __forceinline__ void mesh_nodes(const Ctx &C, int g, double P[4][2])
{
    const int4 q = ((const int4 *)C.mquad)[g];
    const int id[4] = {q.x, q.y, q.z, q.w};
    for (int j = 0; j < 4; ++j) {
        const double2 p = ((const double2 *)C.mxy)[id[j]];
        P[j][0] = p.x;
        P[j][1] = p.y;
    }
}

// Point of the bilinear map of a quad at (u, w) and the map's Jacobian (dX/du x dX/dw).
__device__ __forceinline__ double bilinear(const double P[4][2], double u, double w, double X[2])
{
    for (int a = 0; a < 2; ++a)
        X[a] = (1.0 - u) * (1.0 - w) * P[0][a] + u * (1.0 - w) * P[1][a] + u * w * P[2][a] +
               (1.0 - u) * w * P[3][a];
    double du[2], dw[2];
    for (int a = 0; a < 2; ++a) {
        du[a] = (1.0 - w) * (P[1][a] - P[0][a]) + w * (P[2][a] - P[3][a]);
        dw[a] = (1.0 - u) * (P[3][a] - P[0][a]) + u * (P[2][a] - P[1][a]);
    }
    return du[0] * dw[1] - du[1] * dw[0];
}

// Free flight (Eq. 4) on a quad mesh by face-to-face tracking, in FP64 on absolute
// coordinates (the stored position is relative to the cell's first node).  Inside the
// convex cell the path leaves through the edge with c.n > 0 (n the outward normal) reached
// first, at d / (c.n) with d the distance to the edge's line (0 if rounding put the point
// just outside; ties to the lower edge; an exit exactly at the remaining time stays).
// Interior edges pass the particle on; OUTFLOW / INFLOW edges remove it; SPECULAR edges
// mirror c; WALL edges re-emit it diffusely about the edge's unit normal (the wall sums
// taking that normal).  kMaxBounce reflections and kMaxCross crossings and mirrorings
// together are the caps (the particle then stops where it is), so the loop always ends.  Returns the new global cell, or -1.
template <typename P>
__device__ inline int move_mesh(const Ctx &C, const CaseDev &cs, int g, P xr[3], P v[3], int64_t &id,
                                IdSrc idsrc, double t, uint32_t step, MoveStats &ms, double *surf)
{
    double Pn[4][2];
    mesh_nodes(C, g, Pn);
    double X[2] = {Pn[0][0] + (double)xr[0], Pn[0][1] + (double)xr[1]};
    double V[3] = {(double)v[0], (double)v[1], (double)v[2]};
    int bounce = 0, cross = 0;
    for (;;) {
        double tmin = t;
        int jmin = -1;
        for (int j = 0; j < 4; ++j) {
            const double *A = Pn[j], *B = Pn[(j + 1) & 3];
            const double ex = B[0] - A[0], ey = B[1] - A[1];
            const double vn = V[0] * ey - V[1] * ex;
            if (!(vn > 0.0)) continue;
            const double d = (A[0] - X[0]) * ey - (A[1] - X[1]) * ex;
            double tj = d / vn;
            if (tj < 0.0) tj = 0.0;
            if (tj < tmin) { tmin = tj; jmin = j; }
        }
        if (jmin < 0) {
            X[0] = X[0] + V[0] * t;
            X[1] = X[1] + V[1] * t;
            break;
        }
        X[0] = X[0] + V[0] * tmin;
        X[1] = X[1] + V[1] * tmin;
        t = t - tmin;
        const int nb = C.mnbr[4 * (size_t)g + jmin];
        if (nb >= 0) {
            if (cross == kMaxCross) { ms.capped++; break; }
            ++cross;
            g = nb;
            mesh_nodes(C, g, Pn);
            continue;
        }
        if (nb == HS_EDGE_OUTFLOW || nb == HS_EDGE_INFLOW) return -1;
        const double *A = Pn[jmin], *B = Pn[(jmin + 1) & 3];
        const double ex = B[0] - A[0], ey = B[1] - A[1];
        const double len = sqrt(ex * ex + ey * ey);
        const double nr[3] = {-ey / len, ex / len, 0.0};
        if (nb == HS_EDGE_SPECULAR) {
            if (cross == kMaxCross) { ms.capped++; break; }
            ++cross;
            const double vn = V[0] * nr[0] + V[1] * nr[1];
            V[0] = V[0] - 2.0 * vn * nr[0];
            V[1] = V[1] - 2.0 * vn * nr[1];
            continue;
        }
        ms.hits++;
        if (bounce == kMaxBounce) { ms.capped++; break; }
        if (id < 0) id = idsrc.get();
        const W4 w = draw(cs, kStreamParticle, (uint64_t)id, step, kDrawBounce + bounce);
        ++bounce;
        const double Vin[3] = {V[0], V[1], V[2]};
        diffuse_reflect_n(C.gas, cs, nr, w, V);
        if (surf) surface_hit_n(C.gas, cs, nr, Vin, V, surf);
    }
    xr[0] = (P)(X[0] - Pn[0][0]);
    xr[1] = (P)(X[1] - Pn[0][1]);
    for (int a = 0; a < 3; ++a) v[a] = (P)V[a];
    return g;
}

// Hexahedra: nodes 0-3 the bottom face counter-clockwise seen from above, 4-7 above them;
// face f has the nodes kHexFace[f], counter-clockwise seen from outside.
__constant__ const int kHexFace[6][4] = {{0, 3, 2, 1}, {4, 5, 6, 7}, {0, 1, 5, 4},
                                         {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};

// The eight nodes of global hexahedron g.
__device__ __forceinline__ void hex_nodes(const Ctx &C, int g, double P[8][3])
{
    const int4 q0 = ((const int4 *)C.hnode)[2 * (size_t)g], q1 = ((const int4 *)C.hnode)[2 * (size_t)g + 1];
    const int id[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    for (int j = 0; j < 8; ++j)
        for (int a = 0; a < 3; ++a) P[j][a] = C.hxyz[3 * (size_t)id[j] + a];
}

// Face f: its first node A and nf = (P2 - P0) x (P3 - P1), the outward normal times twice the
// area of a planar face (0 for a face collapsed to a segment).
__device__ __forceinline__ void hex_face(const double P[8][3], int f, const double *&A, double nf[3])
{
    const double *P0 = P[kHexFace[f][0]], *P1 = P[kHexFace[f][1]], *P2 = P[kHexFace[f][2]], *P3 = P[kHexFace[f][3]];
    A = P0;
    const double d1[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
    const double d2[3] = {P3[0] - P1[0], P3[1] - P1[1], P3[2] - P1[2]};
    nf[0] = d1[1] * d2[2] - d1[2] * d2[1];
    nf[1] = d1[2] * d2[0] - d1[0] * d2[2];
    nf[2] = d1[0] * d2[1] - d1[1] * d2[0];
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Face-to-face tracking through hexahedra with planar faces: as move_mesh, over the six faces
// (a face collapsed to a segment is never left through), the sphere's tangent frame for wall
// re-emission.  Position stored relative to the cell's node 0.  Returns the new global cell
// or -1.
template <typename P>
__device__ inline int move_hex(const Ctx &C, const CaseDev &cs, int g, P xr[3], P v[3], int64_t &id,
                               IdSrc idsrc, double t, uint32_t step, MoveStats &ms, double *surf)
{
    double Pn[8][3];
    hex_nodes(C, g, Pn);
    double X[3] = {Pn[0][0] + (double)xr[0], Pn[0][1] + (double)xr[1], Pn[0][2] + (double)xr[2]};
    double V[3] = {(double)v[0], (double)v[1], (double)v[2]};
    int bounce = 0, cross = 0;
    for (;;) {
        double tmin = t;
        int fmin = -1;
        for (int f = 0; f < 6; ++f) {
            const double *A;
            double nf[3];
            hex_face(Pn, f, A, nf);
            const double vn = dot3(V, nf);
            if (!(vn > 0.0)) continue;
            const double d[3] = {A[0] - X[0], A[1] - X[1], A[2] - X[2]};
            double tf = dot3(d, nf) / vn;
            if (tf < 0.0) tf = 0.0;
            if (tf < tmin) { tmin = tf; fmin = f; }
        }
        if (fmin < 0) {
            for (int a = 0; a < 3; ++a) X[a] = X[a] + V[a] * t;
            break;
        }
        for (int a = 0; a < 3; ++a) X[a] = X[a] + V[a] * tmin;
        t = t - tmin;
        const int nb = C.hnbr[8 * (size_t)g + fmin];
        if (nb >= 0) {
            if (cross == kMaxCross) { ms.capped++; break; }
            ++cross;
            g = nb;
            hex_nodes(C, g, Pn);
            continue;
        }
        if (nb == HS_EDGE_OUTFLOW || nb == HS_EDGE_INFLOW) return -1;
        const double *A;
        double nf[3];
        hex_face(Pn, fmin, A, nf);
        const double ln = sqrt(dot3(nf, nf));
        const double nr[3] = {-nf[0] / ln, -nf[1] / ln, -nf[2] / ln};
        if (nb == HS_EDGE_SPECULAR) {
            if (cross == kMaxCross) { ms.capped++; break; }
            ++cross;
            const double vn = dot3(V, nr);
            for (int a = 0; a < 3; ++a) V[a] = V[a] - 2.0 * vn * nr[a];
            continue;
        }
        ms.hits++;
        if (bounce == kMaxBounce) { ms.capped++; break; }
        if (id < 0) id = idsrc.get();
        const W4 w = draw(cs, kStreamParticle, (uint64_t)id, step, kDrawBounce + bounce);
        ++bounce;
        const double Vin[3] = {V[0], V[1], V[2]};
        diffuse_reflect_n(C.gas, cs, nr, w, V);
        if (surf) surface_hit_n(C.gas, cs, nr, Vin, V, surf);
    }
    for (int a = 0; a < 3; ++a) xr[a] = (P)(X[a] - Pn[0][a]);
    for (int a = 0; a < 3; ++a) v[a] = (P)V[a];
    return g;
}

// Flux-weighted normal speed z = beta c_n of a drifting Maxwellian entering a face,
// density ~ z exp(-(z - s)^2) on z > 0, by exact acceptance-rejection (4 words an
// attempt): s >= 0 under |y| e^{-y^2}[y > -s] + s e^{-y^2} (y = z - s), accepting with
// (y + s) / (|y| + s); -3/4 < s < 0 under a Rayleigh envelope accepting with e^{2 z s};
// s <= -3/4 under a Gamma(2, 2|s|) envelope accepting with e^{-z^2}.
__device__ inline double normal_speed(const CaseDev &cs, uint32_t face, uint32_t step, uint32_t base, double s,
                                      int &used)
{
    double z = 0.0;
    if (s >= 0.0) {
        const double e = exp(-s * s);
        const double Ma = 1.0 - 0.5 * e, Mb = s * sqrt(kPi);
        const double pa = Ma / (Ma + Mb);
        z = s > 0.0 ? s : 1.0;
        for (int a = 0; a < kMaxInjectAR; ++a) {
            const W4 w = draw(cs, kStreamFace, face, step, base + (uint32_t)a);
            const double u0 = unid(w.x), u1 = unid(w.y), u2 = unid(w.z), u3 = unid(w.w);
            double y;
            if (u0 < pa) {
                if (u1 * Ma < 0.5) y = sqrt(-log(u2));
                else y = -sqrt(-log(1.0 - u2 * (1.0 - e)));
            } else {
                y = sqrt(-log(u1)) * cospi(2.0 * u2);
                if (y <= -s) continue;
            }
            const double zz = y + s;
            if (zz <= 0.0) continue;
            z = zz;
            if (u3 * (fabs(y) + s) < zz) { used = a + 1; return zz; }
        }
    } else if (s > -0.75) {
        for (int a = 0; a < kMaxInjectAR; ++a) {
            const W4 w = draw(cs, kStreamFace, face, step, base + (uint32_t)a);
            const double zz = sqrt(-log(unid(w.x)));
            z = zz;
            if (unid(w.w) < exp(2.0 * zz * s)) { used = a + 1; return zz; }
        }
    } else {
        for (int a = 0; a < kMaxInjectAR; ++a) {
            const W4 w = draw(cs, kStreamFace, face, step, base + (uint32_t)a);
            const double zz = -(log(unid(w.x)) + log(unid(w.y))) / (-2.0 * s);
            z = zz;
            if (unid(w.w) < exp(-zz * zz)) { used = a + 1; return zz; }
        }
    }
    used = -kMaxInjectAR;
    return z;
}

}  // namespace hsk
