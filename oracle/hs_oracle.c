/*
 * hs_oracle.c -- plain FP64 CPU oracle of the per-time-step particle update of the hybrid
 * SP-Shakhov / DSMC method (Jin, Liu, Yang, Cao, Zhuo, Zhong; arXiv 2506.23917).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU path is checked against.  It is written
 * straight from the paper (Sec. 2.1 DSMC, Sec. 2.2 SP-Shakhov, Sec. 3.1 coupling,
 * Sec. 3.2 Steps 1-6) and from the readings of the paper recorded next to it; it shares
 * no code with the GPU path.  Slow and simple on purpose: one case at a time, one cell at
 * a time, one particle at a time, in array order, all in IEEE double.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11), keyed by the case seed, counter = (entity low 32 bits,
 * entity high 28 bits | stream << 28, step, draw).  Streams: 0 particle (entity = id),
 * 1 cell, 2 inflow face, 3 initialisation (entity = cell).
 */
#include "hs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KB 1.380649e-23               /* Boltzmann constant, J/K                        */
#define PI 3.14159265358979323846
#define MAX_BOUNCE 8                  /* body reflections per particle per step          */
#define MAX_AR 64                     /* Shakhov acceptance-rejection attempts           */
#define MAX_INJ_AR 64                 /* inflow normal-speed attempts                    */
#define MAX_POS_TRY 64                /* initial-position attempts in a cut cell         */
#define SUB 16                        /* sub-cells per axis for cut-cell volumes         */
#define MAX_CROSS 4096                /* mesh edge crossings per particle per step       */

enum { ST_PARTICLE = 0, ST_CELL = 1, ST_FACE = 2, ST_INIT = 3 };
enum { DRAW_RELAX = 0, DRAW_AR = 1, DRAW_BOUNCE = 200, DRAW_INJ_TIME = 300 };

typedef struct {
    int32_t cell;      /* boundary cell, case-local */
    int32_t side;      /* grid: 0..5 = -x,+x,-y,+y,-z,+z; mesh: the cell's edge 0..3 */
    double lambda;     /* expected number of entering particles per step */
} face_t;

typedef struct {
    hso_case p;
    double *region_box;
    hso_state *region_state;
    double *dt_over_tau;
    int64_t ncells;
    double *vol, *sigc_max, *acc, *dt_cell;
    double *lcell;                /* L_cell of Eq. 25 per cell */
    hso_mesh mesh;                /* own copy of a mesh case's arrays */
    double *mxy;
    int32_t *mquad, *mnbr;
    double *surf;                 /* 7 sums per body surface element */
    double dt_cur, dt_next;       /* global step of the coming step; Eq. 26 minimum so far */
    double t_sampled;             /* sum of the global steps of the sampled steps */
    int64_t n_samples;
    int64_t np, cap;
    double *x, *v;
    int32_t *cell;
    int64_t *id;
    int64_t next_id, step;
    int64_t nfaces;
    face_t *faces;
    hso_trace *trace;
    hso_counters cnt;
    /* sort scratch */
    double *x2, *v2;
    int32_t *cell2;
    int64_t *id2;
    int64_t *count;
} ocase;

struct hso_sim {
    hso_gas gas;
    int n_cases;
    ocase *cases;
    int trace_on;
    int failed;
};

/* ------------------------------------------------------------------------------------ */
/* Random numbers                                                                        */
/* ------------------------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds, as defined in Salmon et al. (SC'11): each round multiplies
 * counter words 0 and 2 by two fixed odd constants, and the high halves are mixed with
 * the other two words and the round key; the key is bumped by the golden-ratio and
 * sqrt(3)-1 Weyl constants between rounds. */
void hso_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void hso_draw(uint64_t seed, uint32_t stream, uint64_t entity, uint32_t step,
              uint32_t draw, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = (uint32_t)(entity & 0xffffffffu);
    ctr[1] = (uint32_t)((entity >> 32) & 0x0fffffffu) | (stream << 28);
    ctr[2] = step;
    ctr[3] = draw;
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
    hso_philox4x32_10(ctr, key, out);
}

/* A 32-bit word as a uniform number in the open interval (0,1): (w + 1/2) / 2^32. */
double hso_uniform(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* A 32-bit word as a uniform integer in [0, n): floor(w * n / 2^32). */
uint32_t hso_index(uint32_t w, uint32_t n) { return (uint32_t)(((uint64_t)w * n) >> 32); }

/* ------------------------------------------------------------------------------------ */
/* Gas model (Sec. 4 opening paragraph, Eq. 33; Sec. 2.2 for tau = mu / p)                */
/* ------------------------------------------------------------------------------------ */

/* VHS total cross-section times relative speed (Bird's VHS model, the paper's gas model
 * of Sec. 4): sigma_T = pi d_ref^2 (2 k T_ref / (m_r c_r^2))^(omega-1/2) / Gamma(5/2-omega)
 * with reduced mass m_r = m/2, so sigma_T c_r = K c_r^(2-2 omega). */
static double vhs_K(const hso_gas *g)
{
    return PI * g->d_ref * g->d_ref * pow(4.0 * KB * g->T_ref / g->m, g->omega - 0.5)
           / tgamma(2.5 - g->omega);
}

double hso_sigma_c(const hso_gas *g, double cr)
{
    return vhs_K(g) * pow(cr, 2.0 - 2.0 * g->omega);
}

/* Power-law viscosity with the VHS exponent omega (Sec. 4). */
double hso_viscosity(const hso_gas *g, double T)
{
    return g->mu_ref * pow(T / g->T_ref, g->omega);
}

/* VHS mean free path, Eq. 33. */
double hso_mean_free_path(const hso_gas *g, double n, double T)
{
    return 1.0 / (sqrt(2.0) * PI * g->d_ref * g->d_ref * n * pow(g->T_ref / T, g->omega - 0.5));
}

/* One-way number flux of a drifting Maxwellian through a face with inward unit normal
 * nrm: n (exp(-s^2) + sqrt(pi) s (1 + erf s)) / (2 beta sqrt(pi)), beta = 1/sqrt(2RT),
 * s = beta U.nrm.  (Inflow boundaries are not described in the paper; this is the
 * standard kinetic-theory flux used to feed freestream boundaries.) */
double hso_inflow_number_flux(const hso_gas *g, const hso_state *st, const double nrm[3])
{
    double R = KB / g->m;
    double beta = 1.0 / sqrt(2.0 * R * st->T);
    double s = beta * (st->u[0] * nrm[0] + st->u[1] * nrm[1] + st->u[2] * nrm[2]);
    return st->n * (exp(-s * s) + sqrt(PI) * s * (1.0 + erf(s))) / (2.0 * beta * sqrt(PI));
}

/* Flux-weighted normal speed z = beta c_n > 0, density proportional to
 * z exp(-(z - s)^2), with s = beta U.n the inward drift in thermal units.  Exact
 * acceptance-rejection; each attempt consumes 4 words.
 *  s >= 0: envelope |y| exp(-y^2) [y > -s] + s exp(-y^2), y = z - s, which dominates
 *     (y + s) exp(-y^2) [y > -s].  The first part (mass 1 - exp(-s^2)/2) is sampled
 *     exactly (Rayleigh for y > 0, truncated Rayleigh on (-s, 0)); the second is the
 *     full Gaussian of mass s sqrt(pi), whose draws below -s are rejected.  Keep with
 *     probability (y + s) / (|y| + s).
 *  -3/4 < s < 0: envelope z exp(-z^2) exp(-s^2) (since 2 z s <= 0); z = sqrt(-ln u),
 *     keep with probability exp(2 z s).
 *  s <= -3/4: envelope z exp(-2 |s| z - s^2) (dropping z^2), a Gamma(2, 2|s|) draw,
 *     keep with probability exp(-z^2). */
double hso_sample_normal_speed(double s, const uint32_t *w, int n_attempts, int *used)
{
    double z = 0.0;
    if (s >= 0.0) {
        double e = exp(-s * s);
        double Ma = 1.0 - 0.5 * e;
        double Mb = s * sqrt(PI);
        double pa = Ma / (Ma + Mb);
        z = s > 0.0 ? s : 1.0;
        for (int a = 0; a < n_attempts; ++a) {
            double u0 = hso_uniform(w[4 * a + 0]);
            double u1 = hso_uniform(w[4 * a + 1]);
            double u2 = hso_uniform(w[4 * a + 2]);
            double u3 = hso_uniform(w[4 * a + 3]);
            double y;
            if (u0 < pa) {
                if (u1 * Ma < 0.5)
                    y = sqrt(-log(u2));
                else
                    y = -sqrt(-log(1.0 - u2 * (1.0 - e)));
            } else {
                y = sqrt(-log(u1)) * cos(2.0 * PI * u2);
                if (y <= -s) continue;
            }
            double zz = y + s;
            if (zz <= 0.0) continue;
            z = zz;
            if (u3 * (fabs(y) + s) < zz) {
                *used = a + 1;
                return zz;
            }
        }
    } else if (s > -0.75) {
        for (int a = 0; a < n_attempts; ++a) {
            double zz = sqrt(-log(hso_uniform(w[4 * a + 0])));
            z = zz;
            if (hso_uniform(w[4 * a + 3]) < exp(2.0 * zz * s)) {
                *used = a + 1;
                return zz;
            }
        }
    } else {
        for (int a = 0; a < n_attempts; ++a) {
            double zz = -(log(hso_uniform(w[4 * a + 0])) + log(hso_uniform(w[4 * a + 1]))) / (-2.0 * s);
            z = zz;
            if (hso_uniform(w[4 * a + 3]) < exp(-zz * zz)) {
                *used = a + 1;
                return zz;
            }
        }
    }
    *used = -n_attempts;
    return z;
}

/* ------------------------------------------------------------------------------------ */
/* Geometry                                                                              */
/* ------------------------------------------------------------------------------------ */

static int64_t ncells_of(const hso_case *c)
{
    if (c->mesh) return c->mesh->n_cells;
    if (c->dim == 0) return c->nx;
    int64_t n = c->nx;
    if (c->dim >= 2) n *= c->ny;
    if (c->dim >= 3) n *= c->nz;
    return n;
}

static void cell_ijk(const hso_case *c, int64_t k, int64_t ijk[3])
{
    ijk[0] = ijk[1] = ijk[2] = 0;
    if (c->dim == 0) { ijk[0] = k; return; }
    ijk[0] = k % c->nx;
    if (c->dim >= 2) ijk[1] = (k / c->nx) % c->ny;
    if (c->dim >= 3) ijk[2] = k / ((int64_t)c->nx * c->ny);
}

static int body_axes(const hso_case *c)
{
    return c->body == HSO_BODY_SPHERE ? 3 : 2;
}

/* Is an absolute point strictly inside the body?  (distance^2 < R^2, summed x, y, z) */
static int inside_body(const hso_case *c, const double x[3])
{
    if (c->body == HSO_BODY_NONE) return 0;
    int na = body_axes(c);
    double d2 = 0.0;
    for (int a = 0; a < na; ++a) {
        double d = x[a] - c->body_c[a];
        d2 = d2 + d * d;
    }
    return d2 < c->body_r * c->body_r;
}

/* Cut-cell volume rule: count the 16^dim sub-cell centres
 * lo + (i + (s + 1/2)/16) h that lie outside the body.  Cells whose nearest point is
 * clearly outside (or farthest corner clearly inside) are classified without sampling;
 * the margin makes that exact-equivalent to sampling. */
int64_t hso_cut_count(const hso_case *c, int i, int j, int k)
{
    int dim = c->dim;
    int64_t full = 1;
    for (int a = 0; a < dim; ++a) full *= SUB;
    if (c->body == HSO_BODY_NONE || dim == 0) return full;
    int64_t ijk[3] = { i, j, k };
    int na = body_axes(c);
    double near2 = 0.0, far2 = 0.0;
    for (int a = 0; a < na; ++a) {
        double blo = c->lo[a] + (double)ijk[a] * c->h[a];
        double bhi = c->lo[a] + (double)(ijk[a] + 1) * c->h[a];
        double dn = 0.0;
        if (c->body_c[a] < blo) dn = blo - c->body_c[a];
        else if (c->body_c[a] > bhi) dn = c->body_c[a] - bhi;
        double df = fabs(blo - c->body_c[a]);
        if (fabs(bhi - c->body_c[a]) > df) df = fabs(bhi - c->body_c[a]);
        near2 = near2 + dn * dn;
        far2 = far2 + df * df;
    }
    double R2 = c->body_r * c->body_r;
    if (near2 > R2 * (1.0 + 1e-9)) return full;
    if (far2 < R2 * (1.0 - 1e-9)) return 0;
    int64_t out = 0;
    int s2max = dim >= 3 ? SUB : 1;
    int s1max = dim >= 2 ? SUB : 1;
    for (int s2 = 0; s2 < s2max; ++s2)
        for (int s1 = 0; s1 < s1max; ++s1)
            for (int s0 = 0; s0 < SUB; ++s0) {
                int sub[3] = { s0, s1, s2 };
                double p[3] = { 0.0, 0.0, 0.0 };
                for (int a = 0; a < dim; ++a)
                    p[a] = c->lo[a] + ((double)ijk[a] + ((double)sub[a] + 0.5) / SUB) * c->h[a];
                if (!inside_body(c, p)) ++out;
            }
    return out;
}

/* Node j (taken mod 4) of mesh cell k. */
static void mesh_node(const hso_mesh *m, int64_t k, int j, double P[2])
{
    int32_t n = m->quad[4 * k + (j & 3)];
    P[0] = m->xy[2 * n];
    P[1] = m->xy[2 * n + 1];
}

/* z component of the cross product of (a1 - a0) and (b1 - b0). */
static double cross_d(const double a0[2], const double a1[2], const double b0[2], const double b1[2])
{
    return (a1[0] - a0[0]) * (b1[1] - b0[1]) - (a1[1] - a0[1]) * (b1[0] - b0[0]);
}

/* Area of the convex quad (two triangles from node 0) and its longest edge. */
static void mesh_cell_geometry(const hso_mesh *m, int64_t k, double *area, double *longest)
{
    double P[4][2];
    for (int j = 0; j < 4; ++j) mesh_node(m, k, j, P[j]);
    *area = 0.5 * (cross_d(P[0], P[1], P[0], P[2]) + cross_d(P[0], P[2], P[0], P[3]));
    double lmax = 0.0;
    for (int j = 0; j < 4; ++j) {
        double ex = P[(j + 1) & 3][0] - P[j][0], ey = P[(j + 1) & 3][1] - P[j][1];
        double l = sqrt(ex * ex + ey * ey);
        if (l > lmax) lmax = l;
    }
    *longest = lmax;
}

/* Hexahedra (3-D meshes): nodes 0-3 the bottom quad, counter-clockwise seen from above, nodes
 * 4-7 above them; face f has the nodes HEX_FACE[f], counter-clockwise seen from outside. */
static const int HEX_FACE[6][4] = { { 0, 3, 2, 1 }, { 4, 5, 6, 7 }, { 0, 1, 5, 4 },
                                    { 1, 2, 6, 5 }, { 2, 3, 7, 6 }, { 3, 0, 4, 7 } };

static void hex_node(const hso_mesh *m, int64_t k, int j, double P[3])
{
    int32_t n = m->quad[8 * k + j];
    for (int a = 0; a < 3; ++a) P[a] = m->xy[3 * n + a];
}

/* Face f of hexahedron k: its first node A and the cross product of its diagonals,
 * nf = (P2 - P0) x (P3 - P1), which for a planar face is the outward normal times twice its
 * area (a face collapsed to a segment gives 0). */
static void hex_face(const hso_mesh *m, int64_t k, int f, double A[3], double nf[3])
{
    double P[4][3];
    for (int j = 0; j < 4; ++j) hex_node(m, k, HEX_FACE[f][j], P[j]);
    double d1[3], d2[3];
    for (int a = 0; a < 3; ++a) {
        A[a] = P[0][a];
        d1[a] = P[2][a] - P[0][a];
        d2[a] = P[3][a] - P[1][a];
    }
    nf[0] = d1[1] * d2[2] - d1[2] * d2[1];
    nf[1] = d1[2] * d2[0] - d1[0] * d2[2];
    nf[2] = d1[0] * d2[1] - d1[1] * d2[0];
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Volume as six pyramids from the mean of the nodes, and the largest face area. */
static void hex_geometry(const hso_mesh *m, int64_t k, double *vol, double *amax)
{
    double xc[3] = { 0.0, 0.0, 0.0 }, P[3];
    for (int j = 0; j < 8; ++j) {
        hex_node(m, k, j, P);
        for (int a = 0; a < 3; ++a) xc[a] = xc[a] + P[a];
    }
    for (int a = 0; a < 3; ++a) xc[a] = 0.125 * xc[a];
    double v = 0.0, am = 0.0;
    for (int f = 0; f < 6; ++f) {
        double A[3], nf[3], d[3];
        hex_face(m, k, f, A, nf);
        for (int a = 0; a < 3; ++a) d[a] = A[a] - xc[a];
        v = v + dot3(d, nf) / 6.0;
        double ar = 0.5 * sqrt(dot3(nf, nf));
        if (ar > am) am = ar;
    }
    *vol = v;
    *amax = am;
}

/* Eq. 25's L_cell (reading: the cell's thickness): the smallest edge of a grid cell; a mesh
 * quad's area over its longest edge, which is the same for a rectangle. */
static double cell_length(const hso_case *c, int64_t k)
{
    if (c->mesh && c->dim == 3) {
        double v, am;
        hex_geometry(c->mesh, k, &v, &am);
        return v / am;                  /* volume over the largest face: a box's smallest edge */
    }
    if (c->mesh) {
        double a, l;
        mesh_cell_geometry(c->mesh, k, &a, &l);
        return a / l;
    }
    double L = c->h[0];
    for (int a = 1; a < c->dim; ++a) if (c->h[a] < L) L = c->h[a];
    return L;
}

static double cell_volume(const hso_case *c, int64_t k)
{
    if (c->mesh && c->dim == 3) {
        double v, am;
        hex_geometry(c->mesh, k, &v, &am);
        return v;
    }
    if (c->mesh) {
        double a, l;
        mesh_cell_geometry(c->mesh, k, &a, &l);
        return a * c->h[2];
    }
    double full = c->h[0] * c->h[1] * c->h[2];
    if (c->dim == 0 || c->body == HSO_BODY_NONE) return full;
    int64_t ijk[3];
    cell_ijk(c, k, ijk);
    int64_t tot = 1;
    for (int a = 0; a < c->dim; ++a) tot *= SUB;
    int64_t out = hso_cut_count(c, (int)ijk[0], (int)ijk[1], (int)ijk[2]);
    return (double)out / (double)tot * full;
}

/* ------------------------------------------------------------------------------------ */
/* Maxwellian sampling, Eq. 17                                                           */
/* ------------------------------------------------------------------------------------ */

/* Thermal velocity from four uniforms R1..R4 exactly as Eq. 17 writes it. */
static void maxwell_eq17(double T, double R, const uint32_t w[4], double C[3])
{
    double a = sqrt(2.0 * R * T);
    double r1 = hso_uniform(w[0]), r2 = hso_uniform(w[1]);
    double r3 = hso_uniform(w[2]), r4 = hso_uniform(w[3]);
    C[0] = a * cos(2.0 * PI * r1) * sqrt(-log(r2));
    C[1] = a * cos(2.0 * PI * r3) * sqrt(-log(r4));
    C[2] = a * sin(2.0 * PI * r3) * sqrt(-log(r4));
}

/* ------------------------------------------------------------------------------------ */
/* Creation / destruction                                                                */
/* ------------------------------------------------------------------------------------ */

/* A mesh must hold convex counter-clockwise quads whose node ids are in range, and every
 * edge must name a neighbour that names it back over the same two nodes, or a boundary
 * code (WALL edges need body_T, INFLOW edges an inflow state). */
static int validate_mesh(const hso_case *c)
{
    const hso_mesh *m = c->mesh;
    if (c->dim != 2 || m->n_cells <= 0 || m->n_nodes <= 0 || !m->xy || !m->quad || !m->nbr)
        return HSO_EARG;
    if (c->body == HSO_BODY_SPHERE) return HSO_EARG;
    for (int64_t k = 0; k < m->n_cells; ++k) {
        for (int j = 0; j < 4; ++j) {
            int32_t n = m->quad[4 * k + j];
            if (n < 0 || n >= m->n_nodes) return HSO_EARG;
        }
        double P[4][2];
        for (int j = 0; j < 4; ++j) mesh_node(m, k, j, P[j]);
        for (int j = 0; j < 4; ++j)
            if (!(cross_d(P[j], P[(j + 1) & 3], P[(j + 1) & 3], P[(j + 2) & 3]) > 0.0)) return HSO_EARG;
        for (int j = 0; j < 4; ++j) {
            int32_t nb = m->nbr[4 * k + j];
            if (nb >= 0) {
                if (nb >= m->n_cells) return HSO_EARG;
                int back = 0;
                for (int i = 0; i < 4; ++i)
                    if (m->nbr[4 * (int64_t)nb + i] == (int32_t)k &&
                        m->quad[4 * (int64_t)nb + i] == m->quad[4 * k + ((j + 1) & 3)] &&
                        m->quad[4 * (int64_t)nb + ((i + 1) & 3)] == m->quad[4 * k + j]) back = 1;
                if (!back) return HSO_EARG;
            } else if (nb == HSO_EDGE_WALL) {
                if (!(c->body_T > 0.0)) return HSO_EARG;
            } else if (nb == HSO_EDGE_INFLOW) {
                if (!(c->inflow.T > 0.0) || c->inflow.n < 0.0) return HSO_EARG;
            } else if (nb != HSO_EDGE_OUTFLOW && nb != HSO_EDGE_SPECULAR) {
                return HSO_EARG;
            }
        }
    }
    if (c->n_surf > 0 && (c->body != HSO_BODY_CYLINDER || !(c->body_r > 0.0))) return HSO_EARG;
    return HSO_OK;
}

/* A hexahedral mesh: node ids in range, planar faces (a face may collapse to a triangle or a
 * segment), every node on the inner side of every face (convex cells) and a positive volume;
 * neighbours name each other across faces with the same four nodes; boundary codes as for
 * quads.  Tolerances are 1e-9 of the cell's size. */
static int validate_hex(const hso_case *c)
{
    const hso_mesh *m = c->mesh;
    if (m->n_cells <= 0 || m->n_nodes <= 0 || !m->xy || !m->quad || !m->nbr) return HSO_EARG;
    if (c->body == HSO_BODY_CYLINDER) return HSO_EARG;
    for (int64_t k = 0; k < m->n_cells; ++k) {
        for (int j = 0; j < 8; ++j)
            if (m->quad[8 * k + j] < 0 || m->quad[8 * k + j] >= m->n_nodes) return HSO_EARG;
        double v, am;
        hex_geometry(m, k, &v, &am);
        if (!(v > 0.0)) return HSO_EARG;
        double size = cbrt(v);
        for (int f = 0; f < 6; ++f) {
            double A[3], nf[3];
            hex_face(m, k, f, A, nf);
            double ln = sqrt(dot3(nf, nf));
            if (ln > 0.0) {
                for (int j = 0; j < 8; ++j) {
                    double P[3], d[3];
                    hex_node(m, k, j, P);
                    for (int a = 0; a < 3; ++a) d[a] = A[a] - P[a];
                    double sd = dot3(d, nf) / ln;       /* >= 0 inside, 0 on the face */
                    int on_face = 0;
                    for (int i = 0; i < 4; ++i) on_face |= HEX_FACE[f][i] == j;
                    if (on_face ? fabs(sd) > 1e-9 * size : sd < -1e-9 * size) return HSO_EARG;
                }
            }
            int32_t nb = m->nbr[6 * k + f];
            if (nb >= 0) {
                if (nb >= m->n_cells) return HSO_EARG;
                int back = 0;
                for (int i = 0; i < 6 && !back; ++i) {
                    if (m->nbr[6 * (int64_t)nb + i] != (int32_t)k) continue;
                    int same = 1;
                    for (int a = 0; a < 4; ++a) {
                        int found = 0;
                        for (int b = 0; b < 4; ++b)
                            found |= m->quad[8 * (int64_t)nb + HEX_FACE[i][b]] == m->quad[8 * k + HEX_FACE[f][a]];
                        same &= found;
                    }
                    back = same;
                }
                if (!back) return HSO_EARG;
            } else if (nb == HSO_EDGE_WALL) {
                if (!(c->body_T > 0.0)) return HSO_EARG;
            } else if (nb == HSO_EDGE_INFLOW) {
                if (!(c->inflow.T > 0.0) || c->inflow.n < 0.0) return HSO_EARG;
            } else if (nb != HSO_EDGE_OUTFLOW && nb != HSO_EDGE_SPECULAR) {
                return HSO_EARG;
            }
        }
    }
    if (c->n_surf > 0 && (c->body != HSO_BODY_SPHERE || !(c->body_r > 0.0))) return HSO_EARG;
    return HSO_OK;
}

static int validate_case(const hso_case *c)
{
    if (c->mesh && c->dim == 3) {
        for (int a = 0; a < 3; ++a) if (!(c->h[a] > 0.0)) return HSO_EARG;
        if (!(c->F_N > 0.0) || !(c->T_sigma > 0.0) || c->capacity < 0 || !(c->dt_G > 0.0)) return HSO_EARG;
        return validate_hex(c);
    }
    if (c->mesh) {
        for (int a = 0; a < 3; ++a) if (!(c->h[a] > 0.0)) return HSO_EARG;
        if (!(c->F_N > 0.0) || !(c->T_sigma > 0.0) || c->capacity < 0 || !(c->dt_G > 0.0)) return HSO_EARG;
        return validate_mesh(c);
    }
    if (c->dim < 0 || c->dim > 3) return HSO_EARG;
    if (c->nx <= 0 || (c->dim >= 2 && c->ny <= 0) || (c->dim >= 3 && c->nz <= 0)) return HSO_EARG;
    for (int a = 0; a < 3; ++a) if (!(c->h[a] > 0.0)) return HSO_EARG;
    if (!(c->F_N > 0.0) || !(c->T_sigma > 0.0)) return HSO_EARG;
    if (c->capacity < 0) return HSO_EARG;
    if (c->dim == 0) {
        if (!c->dt_over_tau || c->n_regions < 1 || !c->region_state) return HSO_EARG;
    } else if (!(c->dt_G > 0.0)) return HSO_EARG;
    if (c->body != HSO_BODY_NONE) {
        if (c->body == HSO_BODY_CYLINDER && c->dim < 2) return HSO_EARG;
        if (c->body == HSO_BODY_SPHERE && c->dim < 3) return HSO_EARG;
        if (!(c->body_r > 0.0) || !(c->body_T > 0.0)) return HSO_EARG;
        for (int s = 0; s < 2 * c->dim; ++s) if (c->bc[s] == HSO_BC_SPECULAR) return HSO_EARG;
        for (int a = 0; a < body_axes(c); ++a) {
            double n_a = a == 0 ? c->nx : a == 1 ? c->ny : c->nz;
            if (c->body_c[a] - c->body_r <= c->lo[a]) return HSO_EARG;
            if (c->body_c[a] + c->body_r >= c->lo[a] + n_a * c->h[a]) return HSO_EARG;
        }
    }
    return HSO_OK;
}

static void free_case(ocase *c)
{
    free(c->region_box); free(c->region_state); free(c->dt_over_tau);
    free(c->vol); free(c->sigc_max); free(c->acc); free(c->dt_cell);
    free(c->x); free(c->v); free(c->cell); free(c->id);
    free(c->x2); free(c->v2); free(c->cell2); free(c->id2); free(c->count);
    free(c->faces); free(c->trace); free(c->surf);
    free(c->lcell); free(c->mxy); free(c->mquad); free(c->mnbr);
}

static int alloc_particles(ocase *c, int64_t cap)
{
    size_t n = (size_t)(cap > 0 ? cap : 1);
    c->x = calloc(3 * n, sizeof(double));  c->v = calloc(3 * n, sizeof(double));
    c->cell = calloc(n, sizeof(int32_t));  c->id = calloc(n, sizeof(int64_t));
    c->x2 = calloc(3 * n, sizeof(double)); c->v2 = calloc(3 * n, sizeof(double));
    c->cell2 = calloc(n, sizeof(int32_t)); c->id2 = calloc(n, sizeof(int64_t));
    if (!c->x || !c->v || !c->cell || !c->id || !c->x2 || !c->v2 || !c->cell2 || !c->id2)
        return HSO_ECAP;
    return HSO_OK;
}

/* Inflow faces, in the order: side -x,+x,-y,+y,-z,+z; within a side the boundary cells in
 * x-fastest order.  A face is an inflow face if its side is HSO_BC_INFLOW and its centre
 * lies inside the slot box on every tangential axis where slot_hi > slot_lo. */
/* Inflow edges of a mesh, in cell order and, within a cell, edge order.  The inward unit
 * normal of edge j (node j -> node j+1 of a counter-clockwise quad) is (-e_y, e_x) / |e|;
 * the face area is |e| times the depth h[2]. */
static int build_mesh_faces(const hso_gas *g, ocase *oc)
{
    const hso_case *c = &oc->p;
    const hso_mesh *m = c->mesh;
    oc->faces = calloc((size_t)m->n_cells * 4, sizeof(face_t));
    if (!oc->faces) return HSO_ECAP;
    for (int64_t k = 0; k < m->n_cells; ++k)
        for (int j = 0; j < 4; ++j) {
            if (m->nbr[4 * k + j] != HSO_EDGE_INFLOW) continue;
            double A[2], B[2];
            mesh_node(m, k, j, A);
            mesh_node(m, k, j + 1, B);
            double ex = B[0] - A[0], ey = B[1] - A[1];
            double len = sqrt(ex * ex + ey * ey);
            double nrm[3] = { -ey / len, ex / len, 0.0 };
            double flux = hso_inflow_number_flux(g, &c->inflow, nrm);
            face_t *f = &oc->faces[oc->nfaces++];
            f->cell = (int32_t)k;
            f->side = j;
            f->lambda = flux * (len * c->h[2]) * c->dt_G / c->F_N;
        }
    return HSO_OK;
}

/* Inflow faces of a hexahedral mesh, in cell and face order: area |nf| / 2, inward unit
 * normal -nf / |nf| (faces collapsed to a segment take no inflow). */
static int build_hex_faces(const hso_gas *g, ocase *oc)
{
    const hso_case *c = &oc->p;
    const hso_mesh *m = c->mesh;
    oc->faces = calloc((size_t)m->n_cells * 6, sizeof(face_t));
    if (!oc->faces) return HSO_ECAP;
    for (int64_t k = 0; k < m->n_cells; ++k)
        for (int f = 0; f < 6; ++f) {
            if (m->nbr[6 * k + f] != HSO_EDGE_INFLOW) continue;
            double A[3], nf[3];
            hex_face(m, k, f, A, nf);
            double ln = sqrt(dot3(nf, nf));
            if (!(ln > 0.0)) continue;
            double nrm[3] = { -nf[0] / ln, -nf[1] / ln, -nf[2] / ln };
            double flux = hso_inflow_number_flux(g, &c->inflow, nrm);
            face_t *fc = &oc->faces[oc->nfaces++];
            fc->cell = (int32_t)k;
            fc->side = f;
            fc->lambda = flux * (0.5 * ln) * c->dt_G / c->F_N;
        }
    return HSO_OK;
}

static int build_faces(const hso_gas *g, ocase *oc)
{
    const hso_case *c = &oc->p;
    oc->nfaces = 0;
    if (c->mesh && c->dim == 3) return build_hex_faces(g, oc);
    if (c->mesh) return build_mesh_faces(g, oc);
    if (c->dim == 0) return HSO_OK;
    int64_t n[3] = { c->nx, c->dim >= 2 ? c->ny : 1, c->dim >= 3 ? c->nz : 1 };
    int64_t maxf = 0;
    for (int s = 0; s < 2 * c->dim; ++s) {
        int a = s / 2;
        maxf += ncells_of(c) / n[a];
    }
    oc->faces = calloc((size_t)(maxf > 0 ? maxf : 1), sizeof(face_t));
    if (!oc->faces) return HSO_ECAP;
    for (int s = 0; s < 2 * c->dim; ++s) {
        if (c->bc[s] != HSO_BC_INFLOW) continue;
        int a = s / 2;
        double nrm[3] = { 0.0, 0.0, 0.0 };
        nrm[a] = (s % 2 == 0) ? 1.0 : -1.0;
        double flux = hso_inflow_number_flux(g, &c->inflow, nrm);
        double area = 1.0;
        for (int t = 0; t < 3; ++t) if (t != a) area *= c->h[t];
        double lam = flux * area * c->dt_G / c->F_N;
        for (int64_t k = 0; k < ncells_of(c); ++k) {
            int64_t ijk[3];
            cell_ijk(c, k, ijk);
            if (ijk[a] != ((s % 2 == 0) ? 0 : n[a] - 1)) continue;
            int ok = 1;
            for (int t = 0; t < c->dim; ++t) {
                if (t == a || !(c->slot_hi[t] > c->slot_lo[t])) continue;
                double ctr = c->lo[t] + ((double)ijk[t] + 0.5) * c->h[t];
                if (!(ctr >= c->slot_lo[t] && ctr < c->slot_hi[t])) ok = 0;
            }
            if (!ok) continue;
            face_t *f = &oc->faces[oc->nfaces++];
            f->cell = (int32_t)k;
            f->side = s;
            f->lambda = lam;
        }
    }
    return HSO_OK;
}

int hso_create(const hso_gas *gas, const hso_case *cases, int n_cases, int trace,
               hso_sim **out)
{
    if (!gas || !cases || n_cases <= 0 || !out) return HSO_EARG;
    if (!(gas->m > 0.0) || !(gas->d_ref > 0.0) || !(gas->T_ref > 0.0) || !(gas->mu_ref > 0.0))
        return HSO_EARG;
    for (int i = 0; i < n_cases; ++i) {
        int e = validate_case(&cases[i]);
        if (e) return e;
        for (int j = 0; j < i; ++j)
            if (cases[j].seed == cases[i].seed) return HSO_EARG;
    }
    hso_sim *s = calloc(1, sizeof(hso_sim));
    if (!s) return HSO_ECAP;
    s->gas = *gas;
    s->n_cases = n_cases;
    s->trace_on = trace;
    s->cases = calloc((size_t)n_cases, sizeof(ocase));
    if (!s->cases) { free(s); return HSO_ECAP; }
    for (int ci = 0; ci < n_cases; ++ci) {
        ocase *oc = &s->cases[ci];
        oc->p = cases[ci];
        const hso_case *c = &cases[ci];
        int e = HSO_OK;
        if (c->n_regions > 0) {
            oc->region_box = malloc(sizeof(double) * 6 * (size_t)c->n_regions);
            oc->region_state = malloc(sizeof(hso_state) * (size_t)c->n_regions);
            if (c->region_box) memcpy(oc->region_box, c->region_box, sizeof(double) * 6 * (size_t)c->n_regions);
            else memset(oc->region_box, 0, sizeof(double) * 6 * (size_t)c->n_regions);
            memcpy(oc->region_state, c->region_state, sizeof(hso_state) * (size_t)c->n_regions);
        }
        oc->p.region_box = oc->region_box;
        oc->p.region_state = oc->region_state;
        if (c->mesh) {
            const hso_mesh *m = c->mesh;
            /* per node 2 or 3 coordinates; per cell 4 or 8 nodes and 4 or 6 neighbours */
            size_t dn = c->dim == 3 ? 3 : 2, vn = c->dim == 3 ? 8 : 4, fn = c->dim == 3 ? 6 : 4;
            oc->mxy = malloc(sizeof(double) * dn * (size_t)m->n_nodes);
            oc->mquad = malloc(sizeof(int32_t) * vn * (size_t)m->n_cells);
            oc->mnbr = malloc(sizeof(int32_t) * fn * (size_t)m->n_cells);
            if (!oc->mxy || !oc->mquad || !oc->mnbr) { hso_destroy(s); return HSO_ECAP; }
            memcpy(oc->mxy, m->xy, sizeof(double) * dn * (size_t)m->n_nodes);
            memcpy(oc->mquad, m->quad, sizeof(int32_t) * vn * (size_t)m->n_cells);
            memcpy(oc->mnbr, m->nbr, sizeof(int32_t) * fn * (size_t)m->n_cells);
            oc->mesh.n_nodes = m->n_nodes;
            oc->mesh.n_cells = m->n_cells;
            oc->mesh.xy = oc->mxy;
            oc->mesh.quad = oc->mquad;
            oc->mesh.nbr = oc->mnbr;
            oc->p.mesh = &oc->mesh;
        }
        c = &oc->p;
        oc->ncells = ncells_of(c);
        int64_t nc = oc->ncells;
        if (c->dim == 0) {
            oc->dt_over_tau = malloc(sizeof(double) * (size_t)nc);
            memcpy(oc->dt_over_tau, c->dt_over_tau, sizeof(double) * (size_t)nc);
        }
        oc->p.dt_over_tau = oc->dt_over_tau;
        oc->vol = calloc((size_t)nc, sizeof(double));
        oc->sigc_max = calloc((size_t)nc, sizeof(double));
        oc->acc = calloc((size_t)nc * 13, sizeof(double));
        oc->dt_cell = calloc((size_t)nc, sizeof(double));
        oc->lcell = calloc((size_t)nc, sizeof(double));
        oc->count = calloc((size_t)nc + 1, sizeof(int64_t));
        oc->trace = calloc((size_t)nc, sizeof(hso_trace));
        if (!oc->vol || !oc->sigc_max || !oc->acc || !oc->dt_cell || !oc->lcell || !oc->count || !oc->trace)
            e = HSO_ECAP;
        if (c->n_surf < 0 || (c->n_surf > 0 && c->body == HSO_BODY_NONE)) e = HSO_EARG;
        if (!e && c->n_surf > 0) {
            oc->surf = calloc((size_t)c->n_surf * 7, sizeof(double));
            if (!oc->surf) e = HSO_ECAP;
        }
        if (!e) e = alloc_particles(oc, c->capacity);
        if (!e) e = build_faces(gas, oc);
        if (e) { hso_destroy(s); return e; }
        oc->cap = c->capacity;
        oc->dt_cur = c->dt_G;
        oc->dt_next = INFINITY;
        /* initial (sigma_T c_r)_max: the VHS value at c* = 10 sqrt(k T_sigma / m) */
        double sc0 = hso_sigma_c(gas, 10.0 * sqrt(KB * c->T_sigma / gas->m));
        for (int64_t k = 0; k < nc; ++k) {
            oc->vol[k] = cell_volume(c, k);
            oc->lcell[k] = c->dim > 0 ? cell_length(c, k) : 0.0;
            oc->sigc_max[k] = sc0;
            if (c->dim == 0) {
                /* 0-D: the observation step equals the cell's own step r_k tau_0, with
                 * tau_0 = mu(T_0) / (n_0 k T_0) of the nominal state (Eq. 10's tau) */
                const hso_state *st = &c->region_state[0];
                double tau0 = hso_viscosity(gas, st->T) / (st->n * KB * st->T);
                oc->dt_cell[k] = c->dt_over_tau[k] * tau0;
            } else {
                oc->dt_cell[k] = c->dt_G;
            }
        }
    }
    *out = s;
    return HSO_OK;
}

void hso_destroy(hso_sim *s)
{
    if (!s) return;
    for (int i = 0; i < s->n_cases; ++i) free_case(&s->cases[i]);
    free(s->cases);
    free(s);
}

/* ------------------------------------------------------------------------------------ */
/* Step (1): initialisation                                                              */
/* ------------------------------------------------------------------------------------ */

static const hso_state *region_of(const hso_case *c, int64_t k)
{
    if (c->n_regions <= 0) return NULL;
    if (c->dim == 0) return &c->region_state[0];
    int64_t ijk[3];
    double mc[2] = { 0.0, 0.0 };
    double mc3[3] = { 0.0, 0.0, 0.0 };
    if (c->mesh && c->dim == 3) {
        /* a hexahedron's centre: the mean of its eight nodes */
        for (int j = 0; j < 8; ++j) {
            double P[3];
            hex_node(c->mesh, k, j, P);
            for (int a = 0; a < 3; ++a) mc3[a] = mc3[a] + P[a];
        }
        for (int a = 0; a < 3; ++a) mc3[a] = 0.125 * mc3[a];
    } else if (c->mesh) {
        /* a mesh cell's centre: the mean of its four nodes */
        for (int j = 0; j < 4; ++j) {
            double P[2];
            mesh_node(c->mesh, k, j, P);
            mc[0] = mc[0] + P[0];
            mc[1] = mc[1] + P[1];
        }
        mc[0] = 0.25 * mc[0];
        mc[1] = 0.25 * mc[1];
    } else {
        cell_ijk(c, k, ijk);
    }
    for (int r = 0; r < c->n_regions; ++r) {
        const double *b = &c->region_box[6 * r];
        int in = 1;
        for (int a = 0; a < c->dim; ++a) {
            double ctr = (c->mesh && c->dim == 3) ? mc3[a] : c->mesh ? mc[a] : c->lo[a] + ((double)ijk[a] + 0.5) * c->h[a];
            if (!(ctr >= b[a] && ctr < b[3 + a])) in = 0;
        }
        if (in) return &c->region_state[r];
    }
    return NULL;
}

/* Position of the bilinear map of quad k at (u, w): (1-u)(1-w) P0 + u(1-w) P1 + u w P2 +
 * (1-u) w P3, and its Jacobian J = (dX/du) x (dX/dw). */
static double bilinear(const double P[4][2], double u, double w, double X[2])
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

/* Step (1) in a mesh cell: a point uniform in the quad, by acceptance-rejection on the
 * bilinear map: (u, w) uniform, accepted with probability J(u, w) / J_max (J is bilinear,
 * so J_max is its largest corner value); draws as in the grid case (words 0, 1 the
 * coordinates, word 2 the test); after MAX_POS_TRY rejections the map's centre. */
static void mesh_place(const hso_mesh *m, int64_t k, uint64_t seed, int64_t q, double x[3])
{
    double P[4][2], X[2];
    for (int j = 0; j < 4; ++j) mesh_node(m, k, j, P[j]);
    double jmax = 0.0;
    for (int cu = 0; cu < 2; ++cu)
        for (int cw = 0; cw < 2; ++cw) {
            double jc = bilinear(P, (double)cu, (double)cw, X);
            if (jc > jmax) jmax = jc;
        }
    for (int t = 0; t < MAX_POS_TRY; ++t) {
        uint32_t w[4];
        hso_draw(seed, ST_INIT, (uint64_t)k, 0, (uint32_t)(1 + 128 * q + t), w);
        double J = bilinear(P, hso_uniform(w[0]), hso_uniform(w[1]), X);
        if (hso_uniform(w[2]) * jmax < J) {
            x[0] = X[0];
            x[1] = X[1];
            return;
        }
    }
    bilinear(P, 0.5, 0.5, X);
    x[0] = X[0];
    x[1] = X[1];
}

/* Step (1) in a hexahedron: a point uniform in its bounding box (draw words 0-2, as the grid
 * cell's), accepted when it lies on the inner side of every face; after MAX_POS_TRY
 * rejections the mean of the nodes. */
static void hex_place(const hso_mesh *m, int64_t k, uint64_t seed, int64_t q, double x[3])
{
    double lo[3], hi[3], P[3], xc[3] = { 0.0, 0.0, 0.0 };
    for (int j = 0; j < 8; ++j) {
        hex_node(m, k, j, P);
        for (int a = 0; a < 3; ++a) {
            if (j == 0 || P[a] < lo[a]) lo[a] = P[a];
            if (j == 0 || P[a] > hi[a]) hi[a] = P[a];
            xc[a] = xc[a] + P[a];
        }
    }
    for (int t = 0; t < MAX_POS_TRY; ++t) {
        uint32_t w[4];
        hso_draw(seed, ST_INIT, (uint64_t)k, 0, (uint32_t)(1 + 128 * q + t), w);
        double X[3];
        for (int a = 0; a < 3; ++a) X[a] = lo[a] + hso_uniform(w[a]) * (hi[a] - lo[a]);
        int in = 1;
        for (int f = 0; f < 6 && in; ++f) {
            double A[3], nf[3], d[3];
            hex_face(m, k, f, A, nf);
            for (int a = 0; a < 3; ++a) d[a] = A[a] - X[a];
            if (dot3(d, nf) < 0.0) in = 0;
        }
        if (in) {
            for (int a = 0; a < 3; ++a) x[a] = X[a];
            return;
        }
    }
    for (int a = 0; a < 3; ++a) x[a] = 0.125 * xc[a];
}

/* Step (1): particles uniformly at random inside each cell's fluid part, velocities
 * U + C with C from Eq. 17.  N_k = floor(n V_k / F_N + u). Ids run in cell order. */
static int init_case(const hso_gas *g, ocase *oc)
{
    const hso_case *c = &oc->p;
    double R = KB / g->m;
    oc->np = 0;
    oc->next_id = 0;
    oc->step = 0;
    oc->n_samples = 0;
    oc->dt_cur = c->dt_G;
    oc->dt_next = INFINITY;
    oc->t_sampled = 0.0;
    memset(&oc->cnt, 0, sizeof(oc->cnt));
    memset(oc->acc, 0, sizeof(double) * 13 * (size_t)oc->ncells);
    if (oc->surf) memset(oc->surf, 0, sizeof(double) * 7 * (size_t)c->n_surf);
    for (int64_t k = 0; k < oc->ncells; ++k) {
        const hso_state *st = region_of(c, k);
        if (!st || oc->vol[k] <= 0.0 || st->n <= 0.0) continue;
        uint32_t w[4];
        hso_draw(c->seed, ST_INIT, (uint64_t)k, 0, 0, w);
        int64_t N = (int64_t)floor(st->n * oc->vol[k] / c->F_N + hso_uniform(w[0]));
        if (oc->np + N > oc->cap) return HSO_ECAP;
        int64_t ijk[3] = { 0, 0, 0 };
        if (!c->mesh) cell_ijk(c, k, ijk);
        for (int64_t q = 0; q < N; ++q) {
            int64_t i = oc->np++;
            double *x = &oc->x[3 * i];
            x[0] = x[1] = x[2] = 0.0;
            if (c->mesh && c->dim == 3) {
                hex_place(c->mesh, k, c->seed, q, x);
            } else if (c->mesh) {
                mesh_place(c->mesh, k, c->seed, q, x);
            } else if (c->dim > 0) {
                int placed = 0;
                for (int t = 0; t < MAX_POS_TRY && !placed; ++t) {
                    hso_draw(c->seed, ST_INIT, (uint64_t)k, 0, (uint32_t)(1 + 128 * q + t), w);
                    for (int a = 0; a < c->dim; ++a)
                        x[a] = c->lo[a] + ((double)ijk[a] + hso_uniform(w[a])) * c->h[a];
                    placed = !inside_body(c, x);
                }
                if (!placed) {
                    /* centre of the first sub-cell (x-fastest) that lies outside the body */
                    int s2max = c->dim >= 3 ? SUB : 1, s1max = c->dim >= 2 ? SUB : 1;
                    for (int s2 = 0; s2 < s2max && !placed; ++s2)
                        for (int s1 = 0; s1 < s1max && !placed; ++s1)
                            for (int s0 = 0; s0 < SUB && !placed; ++s0) {
                                int sub[3] = { s0, s1, s2 };
                                for (int a = 0; a < c->dim; ++a)
                                    x[a] = c->lo[a] + ((double)ijk[a] + ((double)sub[a] + 0.5) / SUB) * c->h[a];
                                placed = !inside_body(c, x);
                            }
                }
            }
            hso_draw(c->seed, ST_INIT, (uint64_t)k, 0, (uint32_t)(1 + 128 * q + 64), w);
            double C[3];
            maxwell_eq17(st->T, R, w, C);
            for (int a = 0; a < 3; ++a) oc->v[3 * i + a] = st->u[a] + C[a];
            oc->cell[i] = (int32_t)k;
            oc->id[i] = oc->next_id++;
        }
    }
    double sc0 = hso_sigma_c(g, 10.0 * sqrt(KB * c->T_sigma / g->m));
    for (int64_t k = 0; k < oc->ncells; ++k) oc->sigc_max[k] = sc0;
    return HSO_OK;
}

int hso_init_particles(hso_sim *s)
{
    if (!s) return HSO_EARG;
    for (int i = 0; i < s->n_cases; ++i) {
        int e = init_case(&s->gas, &s->cases[i]);
        if (e) { s->failed = e; return e; }
    }
    return HSO_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Step (2): inflow injection and free transport with walls                              */
/* ------------------------------------------------------------------------------------ */

/* Enter new particles through every inflow face (reading: freestream boundaries are fed
 * by the one-way Maxwellian flux; the paper only states that particles leaving the
 * domain are removed).  Count floor(lambda_f + u); each entering particle is placed
 * uniformly on the face, with a flux-weighted normal speed, Gaussian tangential speeds
 * (Eq. 17 form) and a fresh id; it then moves for a uniform fraction of the step. */
/* Inflow through a mesh edge: the same draws as a grid face, in the edge's frame.  n is the
 * inward unit normal, t the in-plane unit tangent (-n_y, n_x) or its opposite, whichever has
 * t_x + t_y >= 0 (for axis-aligned edges this is the grid face's first tangential axis), z
 * the depth axis.  The point runs along +t from the edge end with the smaller t
 * coordinate; c = n z_n / beta + t (U.t + a cos(2 pi R1) sqrt(-ln R2)) +
 * e_z (U_z + a sin(2 pi R1) sqrt(-ln R2)). */
static int inject_mesh(const hso_gas *g, ocase *oc)
{
    const hso_case *c = &oc->p;
    const hso_mesh *m = c->mesh;
    double R = KB / g->m;
    uint32_t st = (uint32_t)oc->step;
    double beta = 1.0 / sqrt(2.0 * R * c->inflow.T);
    for (int64_t f = 0; f < oc->nfaces; ++f) {
        const face_t *fc = &oc->faces[f];
        uint32_t w[4];
        hso_draw(c->seed, ST_FACE, (uint64_t)f, st, 0, w);
        double lam = c->adapt_dt ? fc->lambda * (oc->dt_cur / c->dt_G) : fc->lambda;
        int64_t nf = (int64_t)floor(lam + hso_uniform(w[0]));
        double A[2], B[2];
        mesh_node(m, fc->cell, fc->side, A);
        mesh_node(m, fc->cell, fc->side + 1, B);
        double ex = B[0] - A[0], ey = B[1] - A[1];
        double len = sqrt(ex * ex + ey * ey);
        double nx = -ey / len, ny = ex / len;
        double tx = -ny, ty = nx;
        if (tx + ty < 0.0) { tx = -tx; ty = -ty; }
        const double *S = A, *E = B;
        if (B[0] * tx + B[1] * ty < A[0] * tx + A[1] * ty) { S = B; E = A; }
        double sn = (c->inflow.u[0] * nx + c->inflow.u[1] * ny) * beta;
        double ut = c->inflow.u[0] * tx + c->inflow.u[1] * ty;
        for (int64_t q = 0; q < nf; ++q) {
            if (oc->np >= oc->cap) return HSO_ECAP;
            int64_t i = oc->np++;
            double *x = &oc->x[3 * i], *v = &oc->v[3 * i];
            uint32_t base = (uint32_t)(1 + 128 * q);
            hso_draw(c->seed, ST_FACE, (uint64_t)f, st, base, w);
            double frac = hso_uniform(w[0]);
            x[0] = S[0] + frac * (E[0] - S[0]);
            x[1] = S[1] + frac * (E[1] - S[1]);
            x[2] = 0.0;
            hso_draw(c->seed, ST_FACE, (uint64_t)f, st, base + 1, w);
            double at = sqrt(2.0 * R * c->inflow.T);
            double rr = sqrt(-log(hso_uniform(w[1])));
            double vt = ut + at * cos(2.0 * PI * hso_uniform(w[0])) * rr;
            v[2] = c->inflow.u[2] + at * sin(2.0 * PI * hso_uniform(w[0])) * rr;
            uint32_t ws[4 * MAX_INJ_AR];
            for (int att = 0; att < MAX_INJ_AR; ++att)
                hso_draw(c->seed, ST_FACE, (uint64_t)f, st, base + 2 + (uint32_t)att, &ws[4 * att]);
            int used;
            double z = hso_sample_normal_speed(sn, ws, MAX_INJ_AR, &used);
            if (used < 0) oc->cnt.inject_cap++;
            v[0] = nx * z / beta + tx * vt;
            v[1] = ny * z / beta + ty * vt;
            oc->cell[i] = fc->cell;
            oc->id[i] = oc->next_id++;
            oc->cnt.injected++;
        }
    }
    return HSO_OK;
}

/* Inflow through a hexahedron's face: the grid face's draws in the face's frame.  n is the
 * inward unit normal; the tangents t1, t2 come from the two coordinate axes other than the
 * one n is most aligned with (lower index first), by Gram-Schmidt (for an axis-aligned face:
 * the grid face's two tangential axes).  The point is the face's bilinear map from the corner
 * of smallest t1 + t2 coordinate, u towards its neighbour of larger t1 coordinate, accepted
 * with probability J / J_max (draw words 0, 1 the coordinates, word 2 the test; retries at
 * draws +66 + r).  c = n z_n / beta + t1 (U.t1 + a cos(2 pi R1) sqrt(-ln R2)) +
 * t2 (U.t2 + a sin(2 pi R1) sqrt(-ln R2)). */
static int inject_hex(const hso_gas *g, ocase *oc)
{
    const hso_case *c = &oc->p;
    const hso_mesh *m = c->mesh;
    double R = KB / g->m;
    uint32_t st = (uint32_t)oc->step;
    double beta = 1.0 / sqrt(2.0 * R * c->inflow.T);
    for (int64_t f = 0; f < oc->nfaces; ++f) {
        const face_t *fc = &oc->faces[f];
        uint32_t w[4];
        hso_draw(c->seed, ST_FACE, (uint64_t)f, st, 0, w);
        double lam = c->adapt_dt ? fc->lambda * (oc->dt_cur / c->dt_G) : fc->lambda;
        int64_t nf = (int64_t)floor(lam + hso_uniform(w[0]));
        double P[4][3], A[3], nfv[3];
        for (int j = 0; j < 4; ++j) hex_node(m, fc->cell, HEX_FACE[fc->side][j], P[j]);
        hex_face(m, fc->cell, fc->side, A, nfv);
        double ln = sqrt(dot3(nfv, nfv));
        double n[3] = { -nfv[0] / ln, -nfv[1] / ln, -nfv[2] / ln };
        int ax = 0;
        for (int a = 1; a < 3; ++a) if (fabs(n[a]) > fabs(n[ax])) ax = a;
        int a1 = ax == 0 ? 1 : 0, a2 = ax == 2 ? 1 : 2;
        double t1[3] = { 0.0, 0.0, 0.0 }, t2[3] = { 0.0, 0.0, 0.0 };
        t1[a1] = 1.0;
        t2[a2] = 1.0;
        double p1 = n[a1];
        for (int a = 0; a < 3; ++a) t1[a] = t1[a] - p1 * n[a];
        double l1 = sqrt(dot3(t1, t1));
        for (int a = 0; a < 3; ++a) t1[a] = t1[a] / l1;
        double q2 = n[a2], r2 = t1[a2];
        for (int a = 0; a < 3; ++a) t2[a] = t2[a] - q2 * n[a] - r2 * t1[a];
        double l2 = sqrt(dot3(t2, t2));
        for (int a = 0; a < 3; ++a) t2[a] = t2[a] / l2;
        int o = 0;
        for (int j = 1; j < 4; ++j)
            if (dot3(t1, P[j]) + dot3(t2, P[j]) < dot3(t1, P[o]) + dot3(t2, P[o])) o = j;
        int ju = (o + 1) & 3, jv = (o + 3) & 3;
        if (dot3(t1, P[jv]) > dot3(t1, P[ju])) { int tmp = ju; ju = jv; jv = tmp; }
        const double *Po = P[o], *Pu = P[ju], *Pv = P[jv], *Pw = P[(o + 2) & 3];
        double jmax = 0.0;
        for (int cu = 0; cu < 2; ++cu)
            for (int cv = 0; cv < 2; ++cv) {
                double du[3], dv[3], cr[3];
                for (int a = 0; a < 3; ++a) {
                    du[a] = (1.0 - cv) * (Pu[a] - Po[a]) + cv * (Pw[a] - Pv[a]);
                    dv[a] = (1.0 - cu) * (Pv[a] - Po[a]) + cu * (Pw[a] - Pu[a]);
                }
                cr[0] = du[1] * dv[2] - du[2] * dv[1];
                cr[1] = du[2] * dv[0] - du[0] * dv[2];
                cr[2] = du[0] * dv[1] - du[1] * dv[0];
                double jc = sqrt(dot3(cr, cr));
                if (jc > jmax) jmax = jc;
            }
        double sn = dot3(c->inflow.u, n) * beta;
        double ut1 = dot3(c->inflow.u, t1), ut2 = dot3(c->inflow.u, t2);
        for (int64_t q = 0; q < nf; ++q) {
            if (oc->np >= oc->cap) return HSO_ECAP;
            int64_t i = oc->np++;
            double *x = &oc->x[3 * i], *v = &oc->v[3 * i];
            uint32_t base = (uint32_t)(1 + 128 * q);
            double u = 0.5, vv = 0.5;
            for (int r = 0; r < 32; ++r) {
                hso_draw(c->seed, ST_FACE, (uint64_t)f, st, r == 0 ? base : base + 66 + (uint32_t)r, w);
                double uu = hso_uniform(w[0]), vq = hso_uniform(w[1]);
                double du[3], dv[3], cr[3];
                for (int a = 0; a < 3; ++a) {
                    du[a] = (1.0 - vq) * (Pu[a] - Po[a]) + vq * (Pw[a] - Pv[a]);
                    dv[a] = (1.0 - uu) * (Pv[a] - Po[a]) + uu * (Pw[a] - Pu[a]);
                }
                cr[0] = du[1] * dv[2] - du[2] * dv[1];
                cr[1] = du[2] * dv[0] - du[0] * dv[2];
                cr[2] = du[0] * dv[1] - du[1] * dv[0];
                if (hso_uniform(w[2]) * jmax < sqrt(dot3(cr, cr))) { u = uu; vv = vq; break; }
            }
            for (int a = 0; a < 3; ++a)
                x[a] = (1.0 - u) * (1.0 - vv) * Po[a] + u * (1.0 - vv) * Pu[a] + u * vv * Pw[a] + (1.0 - u) * vv * Pv[a];
            hso_draw(c->seed, ST_FACE, (uint64_t)f, st, base + 1, w);
            double at = sqrt(2.0 * R * c->inflow.T);
            double rr = sqrt(-log(hso_uniform(w[1])));
            double v1 = ut1 + at * cos(2.0 * PI * hso_uniform(w[0])) * rr;
            double v2 = ut2 + at * sin(2.0 * PI * hso_uniform(w[0])) * rr;
            uint32_t ws[4 * MAX_INJ_AR];
            for (int att = 0; att < MAX_INJ_AR; ++att)
                hso_draw(c->seed, ST_FACE, (uint64_t)f, st, base + 2 + (uint32_t)att, &ws[4 * att]);
            int used;
            double z = hso_sample_normal_speed(sn, ws, MAX_INJ_AR, &used);
            if (used < 0) oc->cnt.inject_cap++;
            for (int a = 0; a < 3; ++a) v[a] = n[a] * z / beta + t1[a] * v1 + t2[a] * v2;
            oc->cell[i] = fc->cell;
            oc->id[i] = oc->next_id++;
            oc->cnt.injected++;
        }
    }
    return HSO_OK;
}

static int inject(const hso_gas *g, ocase *oc)
{
    const hso_case *c = &oc->p;
    if (c->mesh && c->dim == 3) return inject_hex(g, oc);
    if (c->mesh) return inject_mesh(g, oc);
    double R = KB / g->m;
    uint32_t st = (uint32_t)oc->step;
    int64_t n[3] = { c->nx, c->dim >= 2 ? c->ny : 1, c->dim >= 3 ? c->nz : 1 };
    double beta = 1.0 / sqrt(2.0 * R * c->inflow.T);
    for (int64_t f = 0; f < oc->nfaces; ++f) {
        const face_t *fc = &oc->faces[f];
        uint32_t w[4];
        hso_draw(c->seed, ST_FACE, (uint64_t)f, st, 0, w);
        /* lambda is per dt_G; an adapted step scales it */
        double lam = c->adapt_dt ? fc->lambda * (oc->dt_cur / c->dt_G) : fc->lambda;
        int64_t nf = (int64_t)floor(lam + hso_uniform(w[0]));
        int a = fc->side / 2;
        double sg = (fc->side % 2 == 0) ? 1.0 : -1.0;
        int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        int64_t ijk[3];
        cell_ijk(c, fc->cell, ijk);
        double sn = sg * c->inflow.u[a] * beta;
        for (int64_t q = 0; q < nf; ++q) {
            if (oc->np >= oc->cap) return HSO_ECAP;
            int64_t i = oc->np++;
            double *x = &oc->x[3 * i], *v = &oc->v[3 * i];
            uint32_t base = (uint32_t)(1 + 128 * q);
            hso_draw(c->seed, ST_FACE, (uint64_t)f, st, base, w);
            x[0] = x[1] = x[2] = 0.0;
            for (int t = 0; t < c->dim; ++t) {
                if (t == a) continue;
                double frac = hso_uniform(t == t1 ? w[0] : w[1]);
                x[t] = c->lo[t] + ((double)ijk[t] + frac) * c->h[t];
            }
            x[a] = (fc->side % 2 == 0) ? c->lo[a] : c->lo[a] + (double)n[a] * c->h[a];
            hso_draw(c->seed, ST_FACE, (uint64_t)f, st, base + 1, w);
            double at = sqrt(2.0 * R * c->inflow.T);
            double rr = sqrt(-log(hso_uniform(w[1])));
            v[t1] = c->inflow.u[t1] + at * cos(2.0 * PI * hso_uniform(w[0])) * rr;
            v[t2] = c->inflow.u[t2] + at * sin(2.0 * PI * hso_uniform(w[0])) * rr;
            uint32_t ws[4 * MAX_INJ_AR];
            for (int att = 0; att < MAX_INJ_AR; ++att)
                hso_draw(c->seed, ST_FACE, (uint64_t)f, st, base + 2 + (uint32_t)att, &ws[4 * att]);
            int used;
            double z = hso_sample_normal_speed(sn, ws, MAX_INJ_AR, &used);
            if (used < 0) oc->cnt.inject_cap++;
            v[a] = sg * z / beta;
            oc->cell[i] = fc->cell;
            oc->id[i] = oc->next_id++;
            oc->cnt.injected++;
        }
    }
    return HSO_OK;
}

/* Time at which the straight path x + c t first meets the body surface, or -1.
 * Cylinder (axis z): x, y components; sphere: x, y, z.  Hit when the start is not
 * inside (q >= 0), the path approaches (b < 0) and the root q / (-b + sqrt(b^2 - a q))
 * does not exceed t. */
static double body_hit(const hso_case *c, const double x[3], const double v[3], double t)
{
    int na = body_axes(c);
    double a = 0.0, b = 0.0, q = 0.0;
    for (int k = 0; k < na; ++k) {
        double d = x[k] - c->body_c[k];
        a = a + v[k] * v[k];
        b = b + d * v[k];
        q = q + d * d;
    }
    q = q - c->body_r * c->body_r;
    if (!(a > 0.0) || q < 0.0 || b >= 0.0) return -1.0;
    double disc = b * b - a * q;
    if (disc < 0.0) return -1.0;
    double th = q / (-b + sqrt(disc));
    return th <= t ? th : -1.0;
}

/* Diffuse reflection with full accommodation at T_w (Step (2), Eq. 30, read with
 * c_n = sqrt(2 R T_w) sqrt(-ln R1): the printed "cos" is spurious); tangential speeds in
 * the Eq. 17 (y, z) form.  Tangent frame: cylinder t1 = (-n_y, n_x, 0), t2 = z; sphere
 * t1 = normalise(e x n) with e the axis of smallest |n_e| (first on ties), t2 = n x t1. */
/* Outward unit normal of the body at the wall point xh. */
static void body_normal(const hso_case *c, const double xh[3], double nrm[3])
{
    int na = body_axes(c);
    double len = 0.0;
    for (int k = 0; k < 3; ++k) nrm[k] = 0.0;
    for (int k = 0; k < na; ++k) { nrm[k] = xh[k] - c->body_c[k]; len = len + nrm[k] * nrm[k]; }
    len = sqrt(len);
    for (int k = 0; k < na; ++k) nrm[k] = nrm[k] / len;
}

/* The same with the wall's unit normal nrm (pointing into the gas) given; a mesh wall and
 * a cylinder use the planar frame. */
static void diffuse_reflect_n(const hso_case *c, double R, const double nrm[3], const uint32_t w[4],
                              double v[3])
{
    double t1[3] = { 0.0, 0.0, 0.0 }, t2[3] = { 0.0, 0.0, 0.0 };
    if ((c->mesh && c->dim == 2) || c->body == HSO_BODY_CYLINDER) {
        t1[0] = -nrm[1]; t1[1] = nrm[0];
        t2[2] = 1.0;
    } else {
        int e = 0;
        if (fabs(nrm[1]) < fabs(nrm[e])) e = 1;
        if (fabs(nrm[2]) < fabs(nrm[e])) e = 2;
        double ev[3] = { 0.0, 0.0, 0.0 };
        ev[e] = 1.0;
        t1[0] = ev[1] * nrm[2] - ev[2] * nrm[1];
        t1[1] = ev[2] * nrm[0] - ev[0] * nrm[2];
        t1[2] = ev[0] * nrm[1] - ev[1] * nrm[0];
        double l1 = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
        for (int k = 0; k < 3; ++k) t1[k] = t1[k] / l1;
        t2[0] = nrm[1] * t1[2] - nrm[2] * t1[1];
        t2[1] = nrm[2] * t1[0] - nrm[0] * t1[2];
        t2[2] = nrm[0] * t1[1] - nrm[1] * t1[0];
    }
    double a = sqrt(2.0 * R * c->body_T);
    double cn = a * sqrt(-log(hso_uniform(w[0])));
    double rr = sqrt(-log(hso_uniform(w[2])));
    double cs = a * cos(2.0 * PI * hso_uniform(w[1])) * rr;
    double ct = a * sin(2.0 * PI * hso_uniform(w[1])) * rr;
    for (int k = 0; k < 3; ++k) v[k] = cn * nrm[k] + cs * t1[k] + ct * t2[k];
}

static void diffuse_reflect(const hso_case *c, double R, const double xh[3], const uint32_t w[4],
                            double v[3])
{
    double nrm[3];
    body_normal(c, xh, nrm);
    diffuse_reflect_n(c, R, nrm, w, v);
}

/* For the wall's outward unit normal nrm: its polar angle th from the upstream stagnation
 * direction s = -x, and the unit tangent of growing th, t = (n cos th - s) / sin th (zero
 * at the poles). */
static void polar_frame(const double nrm[3], double *th, double tan[3])
{
    double ct = -nrm[0];
    if (ct > 1.0) ct = 1.0;
    if (ct < -1.0) ct = -1.0;
    *th = acos(ct);
    double st = sin(*th);
    double sdir[3] = { -1.0, 0.0, 0.0 };
    for (int k = 0; k < 3; ++k) tan[k] = st > 0.0 ? (nrm[k] * ct - sdir[k]) / st : 0.0;
}

/* Step (5) on the wall: the momentum and energy one diffuse reflection gives the body,
 * added to the surface element of the hit point (sampled steps only). */
static void surface_hit(const hso_gas *g, ocase *oc, const double nrm[3], const double vin[3],
                        const double vout[3])
{
    const hso_case *c = &oc->p;
    double tan[3], th;
    polar_frame(nrm, &th, tan);
    int k = (int)floor(th / PI * (double)c->n_surf);
    if (k < 0) k = 0;
    if (k > c->n_surf - 1) k = c->n_surf - 1;
    double w = g->m * c->F_N, dP[3], e_in = 0.0, e_out = 0.0;
    for (int a = 0; a < 3; ++a) {
        dP[a] = w * (vin[a] - vout[a]);
        e_in = e_in + vin[a] * vin[a];
        e_out = e_out + vout[a] * vout[a];
    }
    double *S = &oc->surf[7 * k];
    S[0] = S[0] + 1.0;
    S[1] = S[1] + (dP[0] * nrm[0] + dP[1] * nrm[1] + dP[2] * nrm[2]);
    S[2] = S[2] + (dP[0] * tan[0] + dP[1] * tan[1] + dP[2] * tan[2]);
    S[3] = S[3] + 0.5 * w * (e_in - e_out);
    for (int a = 0; a < 3; ++a) S[4 + a] = S[4 + a] + dP[a];
}

/* Free transport, Eq. 4: x <- x + c t, with the body's diffuse wall, specular domain
 * walls, and removal through open faces (Step (2)).  Returns the new case-local cell, or
 * -1 when the particle has left the domain. */
static int32_t move_particle(const hso_gas *g, ocase *oc, double *x, double *v, int64_t id,
                             double t)
{
    const hso_case *c = &oc->p;
    double R = KB / g->m;
    uint32_t st = (uint32_t)oc->step;
    if (c->body != HSO_BODY_NONE) {
        for (int b = 0;; ++b) {
            double th = body_hit(c, x, v, t);
            if (th < 0.0) break;
            for (int k = 0; k < c->dim; ++k) x[k] = x[k] + v[k] * th;
            t = t - th;
            oc->cnt.wall_hits++;
            if (b == MAX_BOUNCE) { oc->cnt.bounce_cap++; t = 0.0; break; }
            uint32_t w[4];
            hso_draw(c->seed, ST_PARTICLE, (uint64_t)id, st, (uint32_t)(DRAW_BOUNCE + b), w);
            double vin[3] = { v[0], v[1], v[2] };
            diffuse_reflect(c, R, x, w, v);
            if (oc->surf && oc->step >= c->n_steady) {
                double nrm[3];
                body_normal(c, x, nrm);
                surface_hit(g, oc, nrm, vin, v);
            }
        }
    }
    for (int k = 0; k < c->dim; ++k) x[k] = x[k] + v[k] * t;
    int64_t n[3] = { c->nx, c->ny, c->nz };
    int64_t idx[3] = { 0, 0, 0 };
    for (int k = 0; k < c->dim; ++k) {
        double hi = c->lo[k] + (double)n[k] * c->h[k];
        if (x[k] < c->lo[k]) {
            if (c->bc[2 * k] != HSO_BC_SPECULAR) return -1;
            x[k] = 2.0 * c->lo[k] - x[k];
            v[k] = -v[k];
        } else if (x[k] >= hi) {
            if (c->bc[2 * k + 1] != HSO_BC_SPECULAR) return -1;
            x[k] = 2.0 * hi - x[k];
            v[k] = -v[k];
        }
        int64_t i = (int64_t)floor((x[k] - c->lo[k]) / c->h[k]);
        if (i < 0) i = 0;
        if (i > n[k] - 1) i = n[k] - 1;
        idx[k] = i;
    }
    return (int32_t)(idx[0] + (int64_t)c->nx * (idx[1] + (int64_t)c->ny * idx[2]));
}

/* Free transport on a mesh (Eq. 4 with face-to-face tracking): inside its convex cell the
 * particle flies straight; the edge it leaves through is the one with an outward-moving
 * normal (c.n > 0) reached first, at time d / (c.n) with d the distance to the edge's line
 * along n (taken as 0 when rounding puts the particle just outside; ties go to the lower
 * edge index; an exit at exactly the remaining time keeps the particle in the cell).  Across
 * an interior edge the flight continues in the neighbour; OUTFLOW and INFLOW edges remove
 * it; a SPECULAR edge mirrors c about the edge; a WALL edge re-emits it diffusely at body_T
 * about the edge's unit normal (Eq. 30 reading as for the body), the wall sums taking that
 * normal, and the remaining time goes on.  Caps as for the body (MAX_BOUNCE reflections),
 * and MAX_CROSS edge crossings and mirrorings together; a capped particle stops where it
 * is.  Returns the new cell
 * or -1. */
static int32_t move_mesh(const hso_gas *g, ocase *oc, int32_t k, double *x, double *v, int64_t id,
                         double t)
{
    const hso_case *c = &oc->p;
    const hso_mesh *m = c->mesh;
    double R = KB / g->m;
    uint32_t st = (uint32_t)oc->step;
    int bounce = 0, cross = 0;
    for (;;) {
        double tmin = t;
        int jmin = -1;
        for (int j = 0; j < 4; ++j) {
            double A[2], B[2];
            mesh_node(m, k, j, A);
            mesh_node(m, k, j + 1, B);
            double ex = B[0] - A[0], ey = B[1] - A[1];
            double vn = v[0] * ey - v[1] * ex;          /* c . (e_y, -e_x), outward */
            if (!(vn > 0.0)) continue;
            double d = (A[0] - x[0]) * ey - (A[1] - x[1]) * ex;
            double tj = d / vn;
            if (tj < 0.0) tj = 0.0;
            if (tj < tmin) { tmin = tj; jmin = j; }
        }
        if (jmin < 0) {
            x[0] = x[0] + v[0] * t;
            x[1] = x[1] + v[1] * t;
            return k;
        }
        x[0] = x[0] + v[0] * tmin;
        x[1] = x[1] + v[1] * tmin;
        t = t - tmin;
        int32_t nb = m->nbr[4 * (int64_t)k + jmin];
        if (nb >= 0) {
            if (cross == MAX_CROSS) { oc->cnt.bounce_cap++; return k; }
            ++cross;
            k = nb;
            continue;
        }
        if (nb == HSO_EDGE_OUTFLOW || nb == HSO_EDGE_INFLOW) return -1;
        double A[2], B[2];
        mesh_node(m, k, jmin, A);
        mesh_node(m, k, jmin + 1, B);
        double ex = B[0] - A[0], ey = B[1] - A[1];
        double len = sqrt(ex * ex + ey * ey);
        double nrm[3] = { -ey / len, ex / len, 0.0 };     /* into the cell */
        if (nb == HSO_EDGE_SPECULAR) {
            if (cross == MAX_CROSS) { oc->cnt.bounce_cap++; return k; }
            ++cross;
            double vn = v[0] * nrm[0] + v[1] * nrm[1];
            v[0] = v[0] - 2.0 * vn * nrm[0];
            v[1] = v[1] - 2.0 * vn * nrm[1];
            continue;
        }
        oc->cnt.wall_hits++;
        if (bounce == MAX_BOUNCE) { oc->cnt.bounce_cap++; return k; }
        uint32_t w[4];
        hso_draw(c->seed, ST_PARTICLE, (uint64_t)id, st, (uint32_t)(DRAW_BOUNCE + bounce), w);
        ++bounce;
        double vin[3] = { v[0], v[1], v[2] };
        diffuse_reflect_n(c, R, nrm, w, v);
        if (oc->surf && oc->step >= c->n_steady) surface_hit(g, oc, nrm, vin, v);
    }
}

/* Free transport in a hexahedral mesh: as move_mesh, with the six planar faces of the cell
 * (outward normal nf, the diagonals' cross product; faces collapsed to a segment are never
 * left through) and the sphere's tangent frame for wall re-emission. */
static int32_t move_hex(const hso_gas *g, ocase *oc, int32_t k, double *x, double *v, int64_t id,
                        double t)
{
    const hso_case *c = &oc->p;
    const hso_mesh *m = c->mesh;
    double R = KB / g->m;
    uint32_t st = (uint32_t)oc->step;
    int bounce = 0, cross = 0;
    for (;;) {
        double tmin = t;
        int fmin = -1;
        for (int f = 0; f < 6; ++f) {
            double A[3], nf[3];
            hex_face(m, k, f, A, nf);
            double vn = dot3(v, nf);
            if (!(vn > 0.0)) continue;
            double d[3] = { A[0] - x[0], A[1] - x[1], A[2] - x[2] };
            double tf = dot3(d, nf) / vn;
            if (tf < 0.0) tf = 0.0;
            if (tf < tmin) { tmin = tf; fmin = f; }
        }
        if (fmin < 0) {
            for (int a = 0; a < 3; ++a) x[a] = x[a] + v[a] * t;
            return k;
        }
        for (int a = 0; a < 3; ++a) x[a] = x[a] + v[a] * tmin;
        t = t - tmin;
        int32_t nb = m->nbr[6 * (int64_t)k + fmin];
        if (nb >= 0) {
            if (cross == MAX_CROSS) { oc->cnt.bounce_cap++; return k; }
            ++cross;
            k = nb;
            continue;
        }
        if (nb == HSO_EDGE_OUTFLOW || nb == HSO_EDGE_INFLOW) return -1;
        double A[3], nf[3];
        hex_face(m, k, fmin, A, nf);
        double ln = sqrt(dot3(nf, nf));
        double nrm[3] = { -nf[0] / ln, -nf[1] / ln, -nf[2] / ln };     /* into the cell */
        if (nb == HSO_EDGE_SPECULAR) {
            if (cross == MAX_CROSS) { oc->cnt.bounce_cap++; return k; }
            ++cross;
            double vn = dot3(v, nrm);
            for (int a = 0; a < 3; ++a) v[a] = v[a] - 2.0 * vn * nrm[a];
            continue;
        }
        oc->cnt.wall_hits++;
        if (bounce == MAX_BOUNCE) { oc->cnt.bounce_cap++; return k; }
        uint32_t w[4];
        hso_draw(c->seed, ST_PARTICLE, (uint64_t)id, st, (uint32_t)(DRAW_BOUNCE + bounce), w);
        ++bounce;
        double vin[3] = { v[0], v[1], v[2] };
        diffuse_reflect_n(c, R, nrm, w, v);
        if (oc->surf && oc->step >= c->n_steady) surface_hit(g, oc, nrm, vin, v);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Step (3): index particles into cells (stable counting sort)                            */
/* ------------------------------------------------------------------------------------ */

static void sort_by_cell(ocase *oc)
{
    int64_t nc = oc->ncells;
    memset(oc->count, 0, sizeof(int64_t) * (size_t)(nc + 1));
    for (int64_t i = 0; i < oc->np; ++i)
        if (oc->cell[i] >= 0) oc->count[oc->cell[i]]++;
    int64_t run = 0;
    for (int64_t k = 0; k < nc; ++k) { int64_t t = oc->count[k]; oc->count[k] = run; run += t; }
    oc->count[nc] = run;
    int64_t removed = 0;
    for (int64_t i = 0; i < oc->np; ++i) {
        int32_t k = oc->cell[i];
        if (k < 0) { ++removed; continue; }
        int64_t d = oc->count[k]++;
        memcpy(&oc->x2[3 * d], &oc->x[3 * i], 3 * sizeof(double));
        memcpy(&oc->v2[3 * d], &oc->v[3 * i], 3 * sizeof(double));
        oc->cell2[d] = k;
        oc->id2[d] = oc->id[i];
    }
    oc->cnt.removed += removed;
    double *tx = oc->x; oc->x = oc->x2; oc->x2 = tx;
    double *tv = oc->v; oc->v = oc->v2; oc->v2 = tv;
    int32_t *tc = oc->cell; oc->cell = oc->cell2; oc->cell2 = tc;
    int64_t *ti = oc->id; oc->id = oc->id2; oc->id2 = ti;
    oc->np = run;
}

/* ------------------------------------------------------------------------------------ */
/* Step (3) moments, Step (4) collisions                                                 */
/* ------------------------------------------------------------------------------------ */

/* Unbiased estimators of Step (3): U = mean c; T = m sum|C|^2 / (3 k (N-1));
 * Q = n N / ((N-1)(N-2)) sum (1/2) m |C|^2 C with n = N F_N / V (the printed prefactor
 * 1/V is read as the number density n, the third-central-moment k-statistic factor). */
int hso_cell_moments(const hso_gas *g, int64_t N, const double *v, double F_N, double vol,
                     double U[3], double *T, double Q[3])
{
    U[0] = U[1] = U[2] = 0.0; Q[0] = Q[1] = Q[2] = 0.0; *T = 0.0;
    if (N < 1) return HSO_OK;
    for (int64_t i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) U[a] = U[a] + v[3 * i + a];
    for (int a = 0; a < 3; ++a) U[a] = U[a] / (double)N;
    if (N < 2) return HSO_OK;
    double s2 = 0.0, s3[3] = { 0.0, 0.0, 0.0 };
    for (int64_t i = 0; i < N; ++i) {
        double C[3], c2 = 0.0;
        for (int a = 0; a < 3; ++a) { C[a] = v[3 * i + a] - U[a]; c2 = c2 + C[a] * C[a]; }
        s2 = s2 + c2;
        for (int a = 0; a < 3; ++a) s3[a] = s3[a] + c2 * C[a];
    }
    *T = g->m * s2 / (3.0 * KB * (double)(N - 1));
    if (N >= 3 && vol > 0.0) {
        double n = (double)N * F_N / vol;
        double f = n * (double)N / ((double)(N - 1) * (double)(N - 2));
        for (int a = 0; a < 3; ++a) Q[a] = f * 0.5 * g->m * s3[a];
    }
    return HSO_OK;
}

/* Eq. 27-28: with local observation step dt_c and relaxation time tau, the global step
 * dt_G is narrowed proportionally: DSMC gets dt_G (dt_c <= tau) or (tau/dt_c) dt_G, the
 * Shakhov relaxation gets the rest. */
void hso_split(double dt_c, double tau, double dt_G, double *dt_dsmc, double *dt_sbgk)
{
    if (dt_c <= tau) {
        *dt_dsmc = dt_G;
        *dt_sbgk = 0.0;
    } else {
        *dt_dsmc = (tau / dt_c) * dt_G;
        *dt_sbgk = dt_G - *dt_dsmc;
    }
}

/* Eq. 17-18: draw C from the Maxwellian, weight A = 1 + (1-Pr) Q.C/(5 p R T)
 * (C^2/(R T) - 5) (the standard Shakhov polynomial; the printed C^2/(2RT) is read as a
 * typo), accept when A / A_max > R5, else draw again.  After n_attempts rejections the
 * last draw is kept (return value negative). */
int hso_shakhov_sample(const hso_gas *g, double T, double p, const double Q[3], double a_max,
                       const uint32_t *w, int n_attempts, double C[3])
{
    double R = KB / g->m;
    double RT = R * T;
    for (int a = 0; a < n_attempts; ++a) {
        maxwell_eq17(T, R, &w[5 * a], C);
        double c2 = C[0] * C[0] + C[1] * C[1] + C[2] * C[2];
        double qc = Q[0] * C[0] + Q[1] * C[1] + Q[2] * C[2];
        double A = 1.0 + (1.0 - g->Pr) * qc / (5.0 * p * RT) * (c2 / RT - 5.0);
        if (A / a_max > hso_uniform(w[5 * a + 4])) return a + 1;
    }
    return -n_attempts;
}

static void sums4(const double *v, int64_t N, double out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        for (int a = 0; a < 3; ++a) out[a] = out[a] + v[3 * i + a];
        out[3] = out[3] + v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
    }
}

/* Step (4) for one cell: moments, time split, NTC DSMC sub-step (Eq. 5-9), SP-Shakhov
 * sub-step (Eq. 16-18), conservation rescale (Eq. 19); then Step (5) sampling. */
static void collide_cell(const hso_gas *g, ocase *oc, int64_t k, int64_t s0, int64_t N,
                         int trace_on)
{
    const hso_case *c = &oc->p;
    uint32_t st = (uint32_t)oc->step;
    double *v = &oc->v[3 * s0];
    const int64_t *ids = &oc->id[s0];
    double vol = oc->vol[k];
    double R = KB / g->m;
    hso_trace tr;
    memset(&tr, 0, sizeof(tr));
    tr.n = N;
    if (trace_on) sums4(v, N, tr.pre_sum);

    double U[3], T, Q[3];
    hso_cell_moments(g, N, v, c->F_N, vol, U, &T, Q);
    int active = N >= 2 && T > 0.0 && vol > 0.0;
    if (!active && N >= 2) oc->cnt.skipped_cells++;
    if (active) {
        double n = (double)N * c->F_N / vol;
        double p = n * KB * T;
        double tau = hso_viscosity(g, T) / p;
        double dtG = c->dim == 0 ? oc->dt_cell[k] : oc->dt_cur;
        double dtc;
        if (c->dim == 0) {
            dtc = dtG;
        } else {
            /* Eq. 25 */
            double L = oc->lcell[k];
            double um = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
            dtc = L / (um + sqrt(g->gamma * R * T));
        }
        if (c->dim > 0 && dtc < oc->dt_next) oc->dt_next = dtc;     /* Eq. 26 */
        double dtD, dtS;
        hso_split(dtc, tau, dtG, &dtD, &dtS);
        double p_relax = -expm1(-dtS / tau);             /* Eq. 16 */
        tr.T = T; tr.tau = tau; tr.dt_dsmc = dtD; tr.p_relax = p_relax;

        /* NTC (Eq. 5-6): N_col = floor(M + u) candidates; (sigma c)_max is held fixed
         * during the step and raised afterwards to the largest value seen. */
        double scmax = oc->sigc_max[k];
        double M = 0.5 * (double)N * (double)(N - 1) * c->F_N * scmax * dtD / vol;
        uint32_t w[4];
        hso_draw(c->seed, ST_CELL, (uint64_t)k, st, 0, w);
        int64_t ncol = (int64_t)floor(M + hso_uniform(w[0]));
        double obs = 0.0;
        for (int64_t kk = 0; kk < ncol; ++kk) {
            hso_draw(c->seed, ST_CELL, (uint64_t)k, st, (uint32_t)(1 + 2 * kk), w);
            uint32_t i = hso_index(w[0], (uint32_t)N);
            uint32_t j = hso_index(w[1], (uint32_t)(N - 1));
            if (j >= i) ++j;
            double ua = hso_uniform(w[2]);
            double *ci = &v[3 * i], *cj = &v[3 * j];
            double gx = ci[0] - cj[0], gy = ci[1] - cj[1], gz = ci[2] - cj[2];
            double cr = sqrt(gx * gx + gy * gy + gz * gz);
            double sc = hso_sigma_c(g, cr);
            if (sc > obs) obs = sc;
            if (ua < sc / scmax) {
                /* Eq. 7-9: isotropic VHS scattering */
                hso_draw(c->seed, ST_CELL, (uint64_t)k, st, (uint32_t)(2 + 2 * kk), w);
                double cchi = 2.0 * hso_uniform(w[0]) - 1.0;
                double schi = sqrt(1.0 - cchi * cchi);
                double th = 2.0 * PI * hso_uniform(w[1]);
                double om[3] = { cchi, schi * cos(th), schi * sin(th) };
                for (int a = 0; a < 3; ++a) {
                    double sum = ci[a] + cj[a];
                    ci[a] = 0.5 * (sum - cr * om[a]);
                    cj[a] = 0.5 * (sum + cr * om[a]);
                }
                tr.nacc++;
                tr.acc_hash ^= (uint64_t)(kk + 1) * 0x9E3779B97F4A7C15ull;
            }
        }
        tr.ncol = ncol;
        if (obs > oc->sigc_max[k]) oc->sigc_max[k] = obs;
        oc->cnt.candidates += ncol;
        oc->cnt.accepted += tr.nacc;

        /* SP-Shakhov (Eq. 16-18): each particle independently relaxes with probability
         * P = 1 - exp(-dt_sbgk / tau) to a draw from g^S built from the Step (3) moments */
        double a_max = 1.0;
        if (p_relax > 0.0) {
            double qm = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
            a_max = 1.0 + 20.0 * (1.0 - g->Pr) * qm / (p * sqrt(R * T));
            tr.a_max = a_max;
            uint32_t ws[5 * MAX_AR];
            for (int64_t q = 0; q < N; ++q) {
                hso_draw(c->seed, ST_PARTICLE, (uint64_t)ids[q], st, DRAW_RELAX, w);
                if (!(hso_uniform(w[0]) < p_relax)) continue;
                tr.nrelax++;
                for (int a = 0; a < MAX_AR; ++a) {
                    uint32_t w2[4];
                    hso_draw(c->seed, ST_PARTICLE, (uint64_t)ids[q], st, (uint32_t)(DRAW_AR + 2 * a), w2);
                    memcpy(&ws[5 * a], w2, 4 * sizeof(uint32_t));
                    hso_draw(c->seed, ST_PARTICLE, (uint64_t)ids[q], st, (uint32_t)(DRAW_AR + 2 * a + 1), w2);
                    ws[5 * a + 4] = w2[0];
                }
                double C[3];
                int used = hso_shakhov_sample(g, T, p, Q, a_max, ws, MAX_AR, C);
                if (used < 0) { tr.ar_cap++; used = -used; }
                tr.ar_attempts += used;
                for (int a = 0; a < 3; ++a) v[3 * q + a] = U[a] + C[a];
            }
        }
        oc->cnt.relaxed += tr.nrelax;
        oc->cnt.ar_attempts += tr.ar_attempts;
        oc->cnt.ar_cap += tr.ar_cap;

        /* Eq. 19: rescale every particle of the cell, c' = U + (c - U_p) sqrt(T / T_p) */
        double Up[3], Tp, Qp[3];
        hso_cell_moments(g, N, v, c->F_N, vol, Up, &Tp, Qp);
        if (Tp > 0.0) {
            double f = sqrt(T / Tp);
            for (int64_t q = 0; q < N; ++q)
                for (int a = 0; a < 3; ++a) v[3 * q + a] = U[a] + (v[3 * q + a] - Up[a]) * f;
        }
    }

    /* Step (5): time-averaged sampling once step >= n_steady */
    if ((int64_t)oc->step >= c->n_steady) {
        double *A = &oc->acc[13 * k];
        A[0] = A[0] + (double)N;
        for (int64_t q = 0; q < N; ++q) {
            const double *cv = &v[3 * q];
            double c2 = cv[0] * cv[0] + cv[1] * cv[1] + cv[2] * cv[2];
            A[1] = A[1] + cv[0]; A[2] = A[2] + cv[1]; A[3] = A[3] + cv[2];
            A[4] = A[4] + cv[0] * cv[0]; A[5] = A[5] + cv[1] * cv[1]; A[6] = A[6] + cv[2] * cv[2];
            A[7] = A[7] + cv[0] * cv[1]; A[8] = A[8] + cv[0] * cv[2]; A[9] = A[9] + cv[1] * cv[2];
            A[10] = A[10] + c2 * cv[0]; A[11] = A[11] + c2 * cv[1]; A[12] = A[12] + c2 * cv[2];
        }
    }
    if (trace_on) {
        sums4(v, N, tr.post_sum);
        oc->trace[k] = tr;
    }
}

static int step_case(const hso_gas *g, ocase *oc, int trace_on)
{
    const hso_case *c = &oc->p;
    if (c->dim > 0) {
        int64_t n_old = oc->np;
        int e = inject(g, oc);
        if (e) return e;
        for (int64_t i = 0; i < oc->np; ++i) {
            double t = oc->dt_cur;
            if (i >= n_old) {
                uint32_t w[4];
                hso_draw(c->seed, ST_PARTICLE, (uint64_t)oc->id[i], (uint32_t)oc->step, DRAW_INJ_TIME, w);
                t = oc->dt_cur * hso_uniform(w[0]);
            }
            if (c->mesh && c->dim == 3)
                oc->cell[i] = move_hex(g, oc, oc->cell[i], &oc->x[3 * i], &oc->v[3 * i], oc->id[i], t);
            else if (c->mesh)
                oc->cell[i] = move_mesh(g, oc, oc->cell[i], &oc->x[3 * i], &oc->v[3 * i], oc->id[i], t);
            else
                oc->cell[i] = move_particle(g, oc, &oc->x[3 * i], &oc->v[3 * i], oc->id[i], t);
        }
        sort_by_cell(oc);
    } else {
        /* 0-D: no transport; the particles must already be grouped by cell */
        for (int64_t i = 1; i < oc->np; ++i)
            if (oc->cell[i] < oc->cell[i - 1]) return HSO_ESTATE;
        memset(oc->count, 0, sizeof(int64_t) * (size_t)(oc->ncells + 1));
        for (int64_t i = 0; i < oc->np; ++i) oc->count[oc->cell[i]]++;
        int64_t run = 0;
        for (int64_t k = 0; k < oc->ncells; ++k) { run += oc->count[k]; oc->count[k] = run; }
    }
    /* count[k] now holds the end offset of cell k in the grouped array */
    int64_t start = 0;
    for (int64_t k = 0; k < oc->ncells; ++k) {
        int64_t end = oc->count[k];
        collide_cell(g, oc, k, start, end - start, trace_on);
        start = end;
    }
    for (int64_t i = 0; i < oc->np * 3; ++i)
        if (!isfinite(oc->v[i])) return HSO_ENUM;
    if ((int64_t)oc->step >= c->n_steady) {
        oc->n_samples++;
        oc->t_sampled = oc->t_sampled + oc->dt_cur;
    }
    if (c->adapt_dt && c->dim > 0 && isfinite(oc->dt_next)) oc->dt_cur = oc->dt_next;
    oc->dt_next = INFINITY;
    oc->step++;
    return HSO_OK;
}

int hso_step(hso_sim *s, int64_t n)
{
    if (!s) return HSO_EARG;
    if (s->failed) return HSO_ESTATE;
    for (int64_t it = 0; it < n; ++it)
        for (int i = 0; i < s->n_cases; ++i) {
            int e = step_case(&s->gas, &s->cases[i], s->trace_on);
            if (e) { s->failed = e; return e; }
        }
    return HSO_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Step (6): output                                                                      */
/* ------------------------------------------------------------------------------------ */

/* mode 0: time averages of the Step (5) sums: n = F_N sum N / (S V), U = <c>,
 * T = m/(3k) (<|c|^2> - |U|^2), q_i = (1/2) m n (<c_i|c|^2> - 2 U_j <c_i c_j> -
 * U_i <|c|^2> + 2 U_i |U|^2).  mode 1: the Step (3) estimators of the current state. */
int hso_sample_moments(hso_sim *s, int ci, int mode, double *n, double *u3, double *T,
                       double *q3, int64_t *n_samples)
{
    if (!s || ci < 0 || ci >= s->n_cases) return HSO_EARG;
    ocase *oc = &s->cases[ci];
    const hso_gas *g = &s->gas;
    if (n_samples) *n_samples = oc->n_samples;
    if (mode == 0) {
        for (int64_t k = 0; k < oc->ncells; ++k) {
            const double *A = &oc->acc[13 * k];
            double nn = 0.0, U[3] = { 0.0, 0.0, 0.0 }, TT = 0.0, q[3] = { 0.0, 0.0, 0.0 };
            if (A[0] > 0.0 && oc->n_samples > 0 && oc->vol[k] > 0.0) {
                nn = oc->p.F_N * A[0] / ((double)oc->n_samples * oc->vol[k]);
                for (int a = 0; a < 3; ++a) U[a] = A[1 + a] / A[0];
                double cc = (A[4] + A[5] + A[6]) / A[0];
                double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
                TT = g->m / (3.0 * KB) * (cc - uu);
                double cij[3][3] = { { A[4], A[7], A[8] }, { A[7], A[5], A[9] }, { A[8], A[9], A[6] } };
                for (int a = 0; a < 3; ++a) {
                    double uc = 0.0;
                    for (int b = 0; b < 3; ++b) uc = uc + U[b] * cij[a][b] / A[0];
                    q[a] = 0.5 * g->m * nn * (A[10 + a] / A[0] - 2.0 * uc - U[a] * cc + 2.0 * U[a] * uu);
                }
            }
            if (n) n[k] = nn;
            if (T) T[k] = TT;
            for (int a = 0; a < 3; ++a) { if (u3) u3[3 * k + a] = U[a]; if (q3) q3[3 * k + a] = q[a]; }
        }
        return HSO_OK;
    }
    if (mode != 1) return HSO_EARG;
    /* current state: group by cell (the state is sorted after every step) */
    int64_t i0 = 0;
    for (int64_t k = 0; k < oc->ncells; ++k) {
        int64_t i1 = i0;
        while (i1 < oc->np && oc->cell[i1] == k) ++i1;
        double U[3], TT, q[3];
        hso_cell_moments(g, i1 - i0, &oc->v[3 * i0], oc->p.F_N, oc->vol[k], U, &TT, q);
        if (n) n[k] = oc->vol[k] > 0.0 ? (double)(i1 - i0) * oc->p.F_N / oc->vol[k] : 0.0;
        if (T) T[k] = TT;
        for (int a = 0; a < 3; ++a) { if (u3) u3[3 * k + a] = U[a]; if (q3) q3[3 * k + a] = q[a]; }
        i0 = i1;
    }
    if (i0 != oc->np) return HSO_ESTATE;
    return HSO_OK;
}

/* ------------------------------------------------------------------------------------ */
/* State access                                                                          */
/* ------------------------------------------------------------------------------------ */

int64_t hso_num_particles(const hso_sim *s, int c)
{
    if (!s || c < 0 || c >= s->n_cases) return -1;
    return s->cases[c].np;
}

int64_t hso_num_cells(const hso_sim *s, int c)
{
    if (!s || c < 0 || c >= s->n_cases) return -1;
    return s->cases[c].ncells;
}

int64_t hso_num_faces(const hso_sim *s, int c)
{
    if (!s || c < 0 || c >= s->n_cases) return -1;
    return s->cases[c].nfaces;
}

int hso_face_info(const hso_sim *s, int c, int32_t *cell, int32_t *side, double *lambda)
{
    if (!s || c < 0 || c >= s->n_cases) return HSO_EARG;
    const ocase *oc = &s->cases[c];
    for (int64_t f = 0; f < oc->nfaces; ++f) {
        if (cell) cell[f] = oc->faces[f].cell;
        if (side) side[f] = oc->faces[f].side;
        if (lambda) lambda[f] = oc->faces[f].lambda;
    }
    return HSO_OK;
}

int hso_get_state(const hso_sim *s, int c, double *x3, double *v3, int32_t *cell, int64_t *id,
                  int64_t *next_id, int64_t *step)
{
    if (!s || c < 0 || c >= s->n_cases) return HSO_EARG;
    const ocase *oc = &s->cases[c];
    size_t n = (size_t)oc->np;
    if (x3) memcpy(x3, oc->x, 3 * n * sizeof(double));
    if (v3) memcpy(v3, oc->v, 3 * n * sizeof(double));
    if (cell) memcpy(cell, oc->cell, n * sizeof(int32_t));
    if (id) memcpy(id, oc->id, n * sizeof(int64_t));
    if (next_id) *next_id = oc->next_id;
    if (step) *step = oc->step;
    return HSO_OK;
}

int hso_set_state(hso_sim *s, int c, int64_t np, const double *x3, const double *v3,
                  const int32_t *cell, const int64_t *id, int64_t next_id, int64_t step)
{
    if (!s || c < 0 || c >= s->n_cases || np < 0) return HSO_EARG;
    ocase *oc = &s->cases[c];
    if (np > oc->cap) return HSO_ECAP;
    for (int64_t i = 0; i < np; ++i) {
        if (cell[i] < 0 || cell[i] >= oc->ncells) return HSO_EARG;
        for (int a = 0; a < 3; ++a)
            if (!isfinite(v3[3 * i + a]) || (x3 && !isfinite(x3[3 * i + a]))) return HSO_ENUM;
    }
    size_t n = (size_t)np;
    if (x3) memcpy(oc->x, x3, 3 * n * sizeof(double));
    else memset(oc->x, 0, 3 * n * sizeof(double));
    memcpy(oc->v, v3, 3 * n * sizeof(double));
    memcpy(oc->cell, cell, n * sizeof(int32_t));
    memcpy(oc->id, id, n * sizeof(int64_t));
    oc->np = np;
    oc->next_id = next_id;
    oc->step = step;
    s->failed = 0;
    return HSO_OK;
}

int hso_get_cells(const hso_sim *s, int c, double *vol, double *sigc_max, double *acc13,
                  int64_t *n_samples)
{
    if (!s || c < 0 || c >= s->n_cases) return HSO_EARG;
    const ocase *oc = &s->cases[c];
    size_t nc = (size_t)oc->ncells;
    if (vol) memcpy(vol, oc->vol, nc * sizeof(double));
    if (sigc_max) memcpy(sigc_max, oc->sigc_max, nc * sizeof(double));
    if (acc13) memcpy(acc13, oc->acc, 13 * nc * sizeof(double));
    if (n_samples) *n_samples = oc->n_samples;
    return HSO_OK;
}

int hso_set_cells(hso_sim *s, int c, const double *sigc_max, const double *acc13,
                  int64_t n_samples)
{
    if (!s || c < 0 || c >= s->n_cases) return HSO_EARG;
    ocase *oc = &s->cases[c];
    size_t nc = (size_t)oc->ncells;
    if (sigc_max) memcpy(oc->sigc_max, sigc_max, nc * sizeof(double));
    if (acc13) memcpy(oc->acc, acc13, 13 * nc * sizeof(double));
    oc->n_samples = n_samples;
    return HSO_OK;
}

int hso_get_trace(const hso_sim *s, int c, hso_trace *out)
{
    if (!s || c < 0 || c >= s->n_cases || !s->trace_on) return HSO_EARG;
    memcpy(out, s->cases[c].trace, sizeof(hso_trace) * (size_t)s->cases[c].ncells);
    return HSO_OK;
}

int hso_get_counters(const hso_sim *s, int c, hso_counters *out)
{
    if (!s || c < 0 || c >= s->n_cases) return HSO_EARG;
    *out = s->cases[c].cnt;
    return HSO_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Body surface sampling: raw sums and Eq. 35-36 time averages                           */
/* ------------------------------------------------------------------------------------ */

int hso_get_surface(const hso_sim *s, int ci, double *sums7)
{
    if (!s || ci < 0 || ci >= s->n_cases || !sums7) return HSO_EARG;
    const ocase *oc = &s->cases[ci];
    if (!oc->surf) return HSO_EARG;
    memcpy(sums7, oc->surf, sizeof(double) * 7 * (size_t)oc->p.n_surf);
    return HSO_OK;
}

int hso_set_surface(hso_sim *s, int ci, const double *sums7)
{
    if (!s || ci < 0 || ci >= s->n_cases || !sums7) return HSO_EARG;
    ocase *oc = &s->cases[ci];
    if (!oc->surf) return HSO_EARG;
    memcpy(oc->surf, sums7, sizeof(double) * 7 * (size_t)oc->p.n_surf);
    return HSO_OK;
}

/* Element k spans polar angles [th_k, th_k+1), th_k = k pi / n_surf.  Its area: a
 * cylinder's two strips 2 R (th_k+1 - th_k) times the axial length (the unit depth h_z of a
 * 2-D case, nz h_z in 3-D); a sphere's zone 2 pi R^2 (cos th_k - cos th_k+1).  Over S
 * sampled steps of total time t_S (S dt_G for a fixed step): p = -sum dP.n / (A t_S),
 * tau = sum dP.t / (A t_S), q = sum dE / (A t_S), force = sum dP / t_S.  Eq. 35: C_p = (p - p_inf) / (rho U^2 / 2),
 * C_h = q / (rho U^3 / 2) (and C_f = tau / (rho U^2 / 2)); Eq. 36: C_D, C_L = force along
 * the freestream direction u / |u| and along (-u_y, u_x, 0) / |u|, over rho U^2 A_ref / 2 with
 * A_ref = 2 R times the axial length (cylinder) or pi R^2 (sphere). */
int hso_surface_sample(const hso_sim *s, int ci, double *elem8, double *body5, int64_t *n_samples)
{
    if (!s || ci < 0 || ci >= s->n_cases) return HSO_EARG;
    const ocase *oc = &s->cases[ci];
    const hso_case *c = &oc->p;
    if (!oc->surf) return HSO_EARG;
    if (n_samples) *n_samples = oc->n_samples;
    int ns = c->n_surf;
    double R = c->body_r;
    double len = c->dim == 3 ? (double)c->nz * c->h[2] : c->h[2];
    double time = oc->t_sampled;
    const hso_state *f = &c->inflow;
    double U = sqrt(f->u[0] * f->u[0] + f->u[1] * f->u[1] + f->u[2] * f->u[2]);
    double rho = f->n * s->gas.m, pinf = f->n * KB * f->T;
    double qd = 0.5 * rho * U * U;
    double aref = c->body == HSO_BODY_CYLINDER ? 2.0 * R * len : PI * R * R;
    double F[3] = { 0.0, 0.0, 0.0 };
    for (int k = 0; k < ns; ++k) {
        const double *S = &oc->surf[7 * k];
        double t0 = PI * (double)k / (double)ns, t1 = PI * (double)(k + 1) / (double)ns;
        double area = c->body == HSO_BODY_CYLINDER ? 2.0 * R * (t1 - t0) * len
                                                  : 2.0 * PI * R * R * (cos(t0) - cos(t1));
        double p = 0.0, tau = 0.0, q = 0.0;
        if (time > 0.0) {
            p = -S[1] / (area * time);
            tau = S[2] / (area * time);
            q = S[3] / (area * time);
            for (int a = 0; a < 3; ++a) F[a] = F[a] + S[4 + a] / time;
        }
        if (elem8) {
            double *E = &elem8[8 * k];
            E[0] = 0.5 * (t0 + t1);
            E[1] = area;
            E[2] = p;
            E[3] = tau;
            E[4] = q;
            E[5] = qd > 0.0 ? (p - pinf) / qd : 0.0;
            E[6] = qd > 0.0 ? tau / qd : 0.0;
            E[7] = qd > 0.0 ? q / (qd * U) : 0.0;
        }
    }
    if (body5) {
        for (int a = 0; a < 3; ++a) body5[a] = F[a];
        double drag = 0.0, lift = 0.0;
        if (U > 0.0) {
            drag = (F[0] * f->u[0] + F[1] * f->u[1] + F[2] * f->u[2]) / U;
            lift = (-F[0] * f->u[1] + F[1] * f->u[0]) / U;
        }
        body5[3] = qd > 0.0 ? drag / (qd * aref) : 0.0;
        body5[4] = qd > 0.0 ? lift / (qd * aref) : 0.0;
    }
    return HSO_OK;
}

int hso_step_dt(const hso_sim *s, int ci, double *dt_next, double *t_sampled)
{
    if (!s || ci < 0 || ci >= s->n_cases) return HSO_EARG;
    if (dt_next) *dt_next = s->cases[ci].dt_cur;
    if (t_sampled) *t_sampled = s->cases[ci].t_sampled;
    return HSO_OK;
}

int hso_set_step_dt(hso_sim *s, int ci, double dt, double t_sampled)
{
    if (!s || ci < 0 || ci >= s->n_cases || !(dt > 0.0) || !(t_sampled >= 0.0)) return HSO_EARG;
    s->cases[ci].dt_cur = dt;
    s->cases[ci].t_sampled = t_sampled;
    return HSO_OK;
}

int hso_dsmc_ratio(const hso_sim *s, int ci, double *ratio)
{
    if (!s || ci < 0 || ci >= s->n_cases || !ratio) return HSO_EARG;
    const ocase *oc = &s->cases[ci];
    const hso_case *c = &oc->p;
    const hso_gas *g = &s->gas;
    int64_t nc = oc->ncells;
    double *n = malloc(sizeof(double) * (size_t)nc), *u = malloc(sizeof(double) * 3 * (size_t)nc);
    double *T = malloc(sizeof(double) * (size_t)nc);
    if (!n || !u || !T) { free(n); free(u); free(T); return HSO_ECAP; }
    int e = hso_sample_moments((hso_sim *)s, ci, 0, n, u, T, NULL, NULL);
    double R = KB / g->m;
    for (int64_t k = 0; !e && k < nc; ++k) {
        ratio[k] = 0.0;
        if (!(n[k] > 0.0) || !(T[k] > 0.0)) continue;
        double tau = hso_viscosity(g, T[k]) / (n[k] * KB * T[k]);
        double dtc;
        if (c->dim == 0) {
            dtc = oc->dt_cell[k];
        } else {
            const double *U = &u[3 * k];
            dtc = oc->lcell[k] / (sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]) + sqrt(g->gamma * R * T[k]));
        }
        ratio[k] = dtc <= tau ? 1.0 : tau / dtc;
    }
    free(n); free(u); free(T);
    return e;
}
