// hs_runtime.cpp -- host side of the C ABI declared in include/hs.h: case validation,
// inflow-face tables, the workspace layout, initialisation, the step sequence (plain
// launches, a replayed hipGraph, or launches bracketed by HIP events), output and
// checkpoints.  All particle work runs in the kernels of hs_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hs_common.hpp"

using namespace hsk;

namespace {

constexpr double kKB_h = 1.380649e-23;
constexpr double kPi_h = 3.14159265358979323846;
constexpr uint32_t kMagic = 0x48534331u;  // "HSC1"

// Offsets of the device arrays.  The sim's own data (case tables, particle state, per-cell
// state and outputs) come first; the arrays a step only uses as scratch (new cells, slots,
// permutation, scan, tiles, cell records, output staging) follow from scratch_begin.  One
// workspace holds both parts back to back; hs_init_particles_static puts the second part in
// the library's fixed device array instead.
struct Layout {
    size_t total = 0;
    size_t scratch_begin = 0;
    size_t globals, cases, faces, rbox, rstate, dtcell;
    size_t pos[2][3], vel[2][3], cell[2], id[2];
    size_t newcell, slot, perm, work, count, cstart, sigc, acc, vol, facecnt, facestart, scanpart, big, tiles, tilecase, cellrec, surf, trace, out;
    size_t mxy = 0, mquad = 0, mnbr = 0, mgeo = 0, hxyz = 0, hnode = 0, hnbr = 0;
    size_t surf_bytes = 0;
};

struct Plan {
    std::vector<CaseDev> cases;
    std::vector<FaceDev> faces;
    std::vector<double> rbox;
    std::vector<StateDev> rstate;
    std::vector<double> dtcell;     // per global cell, only if some case is 0-D
    // quad meshes of the batch, only if some case has one: node coordinates (global node
    // ids), per global cell the node ids, neighbours (global cells or hs_edge codes) and
    // (volume, L_cell)
    std::vector<double> mxy, mgeo;
    std::vector<int32_t> mquad, mnbr;
    // hexahedral meshes: node coordinates (3 per node), 8 node ids and 8 neighbour words
    // (faces 0-5, 2 unused) per global cell
    std::vector<double> hxyz;
    std::vector<int32_t> hnode, hnbr;
    bool any_quad = false, any_hex = false;
    int64_t ncells = 0, capacity = 0;
    int dim_max = 0;
    bool any_spatial = false, any_0d = false, any_body = false, any_mesh = false;
    GasDev gas;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Length of the first k size-class lists of the dense cells: the list of class j reserves room
// for every cell that can hold more than the class's floor of particles, at most
// capacity / (floor + 1) of the batch's cells.
size_t dense_list_length(int64_t capacity, size_t ncells, int k)
{
    size_t o = 0;
    for (int j = 0; j < k; ++j) {
        const int64_t most = capacity / ((int64_t)dense_class_floor(j, cap_wave()) + 1);
        o += std::min<size_t>(ncells, (size_t)std::max<int64_t>(most, 0));
    }
    return o;
}

double cross2(const double *a0, const double *a1, const double *b0, const double *b1)
{
    return (a1[0] - a0[0]) * (b1[1] - b0[1]) - (a1[1] - a0[1]) * (b1[0] - b0[0]);
}

// A mesh: node ids in range, convex counter-clockwise quads, neighbours that name the cell
// back across the same two nodes, boundary codes with what they need.
constexpr int kHexFaceH[6][4] = {{0, 3, 2, 1}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};

double dot3h(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Face f of a hexahedron with nodes P: first node and the diagonals' cross product.
void hex_face_h(const double P[8][3], int f, const double *&A, double nf[3])
{
    const double *P0 = P[kHexFaceH[f][0]], *P1 = P[kHexFaceH[f][1]], *P2 = P[kHexFaceH[f][2]], *P3 = P[kHexFaceH[f][3]];
    A = P0;
    const double d1[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
    const double d2[3] = {P3[0] - P1[0], P3[1] - P1[1], P3[2] - P1[2]};
    nf[0] = d1[1] * d2[2] - d1[2] * d2[1];
    nf[1] = d1[2] * d2[0] - d1[0] * d2[2];
    nf[2] = d1[0] * d2[1] - d1[1] * d2[0];
}

void hex_nodes_h(const hs_mesh *m, int64_t k, double P[8][3])
{
    for (int j = 0; j < 8; ++j)
        for (int a = 0; a < 3; ++a) P[j][a] = m->xy[3 * (size_t)m->quad[8 * k + j] + a];
}

// Volume (six pyramids from the mean of the nodes) and the largest face area.
void hex_geometry_h(const double P[8][3], double &vol, double &amax)
{
    double xc[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 8; ++j)
        for (int a = 0; a < 3; ++a) xc[a] = xc[a] + P[j][a];
    for (int a = 0; a < 3; ++a) xc[a] = 0.125 * xc[a];
    double v = 0.0, am = 0.0;
    for (int f = 0; f < 6; ++f) {
        const double *A;
        double nf[3];
        hex_face_h(P, f, A, nf);
        const double d[3] = {A[0] - xc[0], A[1] - xc[1], A[2] - xc[2]};
        v = v + dot3h(d, nf) / 6.0;
        const double ar = 0.5 * std::sqrt(dot3h(nf, nf));
        if (ar > am) am = ar;
    }
    vol = v;
    amax = am;
}

// A hexahedral mesh: node ids in range, planar faces, every node on the inner side of every
// face (tolerance 1e-9 of the cell size), positive volume, neighbours across faces with the
// same four nodes, boundary codes with what they need.
bool valid_hex(const hs_case &c, std::string &why)
{
    const hs_mesh *m = c.mesh;
    if (m->n_cells <= 0 || m->n_nodes <= 0 || !m->xy || !m->quad || !m->nbr) { why = "mesh arrays"; return false; }
    if (c.body == HS_BODY_CYLINDER) { why = "a hexahedral mesh has no cylinder"; return false; }
    for (int64_t k = 0; k < m->n_cells; ++k) {
        for (int j = 0; j < 8; ++j)
            if (m->quad[8 * k + j] < 0 || m->quad[8 * k + j] >= m->n_nodes) { why = "mesh node id out of range"; return false; }
        double P[8][3], v, am;
        hex_nodes_h(m, k, P);
        hex_geometry_h(P, v, am);
        if (!(v > 0.0)) { why = "hexahedra must have a positive volume"; return false; }
        const double size = std::cbrt(v);
        for (int f = 0; f < 6; ++f) {
            const double *A;
            double nf[3];
            hex_face_h(P, f, A, nf);
            const double ln = std::sqrt(dot3h(nf, nf));
            if (ln > 0.0) {
                for (int j = 0; j < 8; ++j) {
                    const double d[3] = {A[0] - P[j][0], A[1] - P[j][1], A[2] - P[j][2]};
                    const double sd = dot3h(d, nf) / ln;
                    bool on_face = false;
                    for (int i = 0; i < 4; ++i) on_face |= kHexFaceH[f][i] == j;
                    if (on_face ? std::fabs(sd) > 1e-9 * size : sd < -1e-9 * size) {
                        why = "hexahedra must be convex with planar faces";
                        return false;
                    }
                }
            }
            const int32_t nb = m->nbr[6 * k + f];
            if (nb >= 0) {
                if (nb >= m->n_cells) { why = "mesh neighbour out of range"; return false; }
                bool back = false;
                for (int i = 0; i < 6 && !back; ++i) {
                    if (m->nbr[6 * (int64_t)nb + i] != (int32_t)k) continue;
                    bool same = true;
                    for (int a = 0; a < 4; ++a) {
                        bool found = false;
                        for (int b = 0; b < 4; ++b)
                            found |= m->quad[8 * (int64_t)nb + kHexFaceH[i][b]] == m->quad[8 * k + kHexFaceH[f][a]];
                        same &= found;
                    }
                    back = same;
                }
                if (!back) { why = "mesh neighbours must name each other across the same face"; return false; }
            } else if (nb == HS_EDGE_WALL) {
                if (!(c.body_T > 0)) { why = "WALL faces need body_T"; return false; }
            } else if (nb == HS_EDGE_INFLOW) {
                if (!(c.inflow.T > 0 && c.inflow.n >= 0)) { why = "inflow state"; return false; }
            } else if (nb != HS_EDGE_OUTFLOW && nb != HS_EDGE_SPECULAR) {
                why = "unknown mesh face code";
                return false;
            }
        }
    }
    if (c.n_surf > 0 && (c.body != HS_BODY_SPHERE || !(c.body_r > 0))) {
        why = "hexahedral surface elements need a sphere frame (body_r)";
        return false;
    }
    return true;
}

bool valid_mesh(const hs_case &c, std::string &why)
{
    const hs_mesh *m = c.mesh;
    if (c.dim == 3) return valid_hex(c, why);
    if (c.dim != 2) { why = "a mesh case needs dim 2 or 3"; return false; }
    if (m->n_cells <= 0 || m->n_nodes <= 0 || !m->xy || !m->quad || !m->nbr) { why = "mesh arrays"; return false; }
    if (c.body == HS_BODY_SPHERE) { why = "a mesh case has no sphere"; return false; }
    for (int64_t k = 0; k < m->n_cells; ++k) {
        const int32_t *q = &m->quad[4 * k];
        for (int j = 0; j < 4; ++j)
            if (q[j] < 0 || q[j] >= m->n_nodes) { why = "mesh node id out of range"; return false; }
        for (int j = 0; j < 4; ++j) {
            const double *a = &m->xy[2 * q[j]], *b = &m->xy[2 * q[(j + 1) & 3]], *d = &m->xy[2 * q[(j + 2) & 3]];
            if (!(cross2(a, b, b, d) > 0.0)) { why = "mesh cells must be convex and counter-clockwise"; return false; }
        }
        for (int j = 0; j < 4; ++j) {
            const int32_t nb = m->nbr[4 * k + j];
            if (nb >= 0) {
                if (nb >= m->n_cells) { why = "mesh neighbour out of range"; return false; }
                bool back = false;
                for (int i = 0; i < 4; ++i)
                    if (m->nbr[4 * (int64_t)nb + i] == (int32_t)k && m->quad[4 * (int64_t)nb + i] == q[(j + 1) & 3] &&
                        m->quad[4 * (int64_t)nb + ((i + 1) & 3)] == q[j]) back = true;
                if (!back) { why = "mesh neighbours must name each other across the same edge"; return false; }
            } else if (nb == HS_EDGE_WALL) {
                if (!(c.body_T > 0)) { why = "WALL edges need body_T"; return false; }
            } else if (nb == HS_EDGE_INFLOW) {
                if (!(c.inflow.T > 0 && c.inflow.n >= 0)) { why = "inflow state"; return false; }
            } else if (nb != HS_EDGE_OUTFLOW && nb != HS_EDGE_SPECULAR) {
                why = "unknown mesh edge code";
                return false;
            }
        }
    }
    if (c.n_surf > 0 && (c.body != HS_BODY_CYLINDER || !(c.body_r > 0))) {
        why = "mesh surface elements need a cylinder frame (body_r)";
        return false;
    }
    return true;
}

hs_status validate(const hs_gas *g, const hs_case *cs, int n, std::string &why)
{
    if (!g || !cs || n <= 0) { why = "null gas/cases or no cases"; return HS_ERR_ARG; }
    if (n > kMaxCases) { why = "too many cases"; return HS_ERR_ARG; }
    if (!(g->m > 0) || !(g->d_ref > 0) || !(g->T_ref > 0) || !(g->mu_ref > 0) || !(g->gamma > 1) ||
        !(g->Pr > 0) || !(g->omega > 0.5 && g->omega < 1.5)) {
        why = "invalid gas";
        return HS_ERR_ARG;
    }
    int64_t cells = 0, cap = 0;
    for (int i = 0; i < n; ++i) {
        const hs_case &c = cs[i];
        if (c.mesh) {
            for (int a = 0; a < 3; ++a)
                if (!(c.h[a] > 0)) { why = "cell size"; return HS_ERR_ARG; }
            if (!(c.F_N > 0) || !(c.T_sigma > 0) || c.capacity < 0 || !(c.dt_G > 0)) { why = "F_N/T_sigma/capacity/dt_G"; return HS_ERR_ARG; }
            if (c.n_regions < 0 || (c.n_regions > 0 && (!c.region_state || !c.region_box))) { why = "regions"; return HS_ERR_ARG; }
            if (c.adapt_dt != 0 && c.adapt_dt != 1) { why = "adapt_dt must be 0 or 1"; return HS_ERR_ARG; }
            if (c.n_surf < 0 || c.n_surf > 65536) { why = "n_surf (0..65536)"; return HS_ERR_ARG; }
            if (!valid_mesh(c, why)) return HS_ERR_ARG;
            for (int j = 0; j < i; ++j)
                if (cs[j].seed == c.seed) { why = "cases need distinct seeds"; return HS_ERR_ARG; }
            cells += c.mesh->n_cells;
            cap += c.capacity;
            continue;
        }
        if (c.dim < 0 || c.dim > 3) { why = "dim"; return HS_ERR_ARG; }
        if (c.nx <= 0 || (c.dim >= 2 && c.ny <= 0) || (c.dim >= 3 && c.nz <= 0)) { why = "grid size"; return HS_ERR_ARG; }
        for (int a = 0; a < 3; ++a)
            if (!(c.h[a] > 0)) { why = "cell size"; return HS_ERR_ARG; }
        if (!(c.F_N > 0) || !(c.T_sigma > 0) || c.capacity < 0) { why = "F_N/T_sigma/capacity"; return HS_ERR_ARG; }
        if (c.dim == 0) {
            if (!c.dt_over_tau || c.n_regions < 1 || !c.region_state) { why = "0-D case needs dt_over_tau and a region state"; return HS_ERR_ARG; }
        } else if (!(c.dt_G > 0)) { why = "dt_G"; return HS_ERR_ARG; }
        if (c.n_regions < 0 || (c.n_regions > 0 && (!c.region_state || (c.dim > 0 && !c.region_box)))) { why = "regions"; return HS_ERR_ARG; }
        for (int s = 0; s < 2 * c.dim; ++s)
            if (c.bc[s] < HS_BC_OUTFLOW || c.bc[s] > HS_BC_INFLOW) { why = "bc"; return HS_ERR_ARG; }
        bool inflow = false;
        for (int s = 0; s < 2 * c.dim; ++s) inflow |= c.bc[s] == HS_BC_INFLOW;
        if (inflow && !(c.inflow.T > 0 && c.inflow.n >= 0)) { why = "inflow state"; return HS_ERR_ARG; }
        if (c.body != HS_BODY_NONE) {
            if (c.body == HS_BODY_CYLINDER && c.dim < 2) { why = "cylinder needs dim >= 2"; return HS_ERR_ARG; }
            if (c.body == HS_BODY_SPHERE && c.dim < 3) { why = "sphere needs dim 3"; return HS_ERR_ARG; }
            if (c.body < 0 || c.body > 2 || !(c.body_r > 0) || !(c.body_T > 0)) { why = "body"; return HS_ERR_ARG; }
            for (int s = 0; s < 2 * c.dim; ++s)
                if (c.bc[s] == HS_BC_SPECULAR) { why = "specular walls with a body"; return HS_ERR_ARG; }
            const int na = c.body == HS_BODY_SPHERE ? 3 : 2;
            const int nn[3] = {c.nx, c.ny, c.nz};
            for (int a = 0; a < na; ++a)
                if (!(c.body_c[a] - c.body_r > c.lo[a]) || !(c.body_c[a] + c.body_r < c.lo[a] + nn[a] * c.h[a])) {
                    why = "body must lie strictly inside the domain";
                    return HS_ERR_ARG;
                }
        }
        if (c.adapt_dt != 0 && c.adapt_dt != 1) { why = "adapt_dt must be 0 or 1"; return HS_ERR_ARG; }
        if (c.n_surf < 0 || c.n_surf > 65536 || (c.n_surf > 0 && c.body == HS_BODY_NONE)) {
            why = "n_surf (0..65536, needs a body)";
            return HS_ERR_ARG;
        }
        for (int j = 0; j < i; ++j)
            if (cs[j].seed == c.seed) { why = "cases need distinct seeds"; return HS_ERR_ARG; }
        int64_t nc = c.nx;
        if (c.dim >= 2) nc *= c.ny;
        if (c.dim >= 3) nc *= c.nz;
        cells += nc;
        cap += c.capacity;
    }
    if (cells >= (1ll << 31) - 1 || cap >= (1ll << 31) - 64) { why = "batch too large for 32-bit indices"; return HS_ERR_ARG; }
    return HS_OK;
}

double vhs_K(const hs_gas *g)
{
    return kPi_h * g->d_ref * g->d_ref * std::pow(4.0 * kKB_h * g->T_ref / g->m, g->omega - 0.5) /
           std::tgamma(2.5 - g->omega);
}

// One-way number flux of the inflow state through a face with inward normal +-e_a.
double face_flux(const hs_gas *g, const hs_state &st, int a, double sg)
{
    const double R = kKB_h / g->m;
    const double beta = 1.0 / std::sqrt(2.0 * R * st.T);
    double nrm[3] = {0.0, 0.0, 0.0};
    nrm[a] = sg;
    const double s = beta * (st.u[0] * nrm[0] + st.u[1] * nrm[1] + st.u[2] * nrm[2]);
    return st.n * (std::exp(-s * s) + std::sqrt(kPi_h) * s * (1.0 + std::erf(s))) / (2.0 * beta * std::sqrt(kPi_h));
}

// One-way number flux of the inflow state through a face with 3-D inward unit normal nrm.
double edge_flux3(const hs_gas *g, const hs_state &st, const double nrm[3])
{
    const double R = kKB_h / g->m;
    const double beta = 1.0 / std::sqrt(2.0 * R * st.T);
    const double s = beta * (st.u[0] * nrm[0] + st.u[1] * nrm[1] + st.u[2] * nrm[2]);
    return st.n * (std::exp(-s * s) + std::sqrt(kPi_h) * s * (1.0 + std::erf(s))) / (2.0 * beta * std::sqrt(kPi_h));
}

// One-way number flux of the inflow state through a face with inward unit normal nrm.
double edge_flux(const hs_gas *g, const hs_state &st, const double nrm[2])
{
    const double R = kKB_h / g->m;
    const double beta = 1.0 / std::sqrt(2.0 * R * st.T);
    const double s = beta * (st.u[0] * nrm[0] + st.u[1] * nrm[1]);
    return st.n * (std::exp(-s * s) + std::sqrt(kPi_h) * s * (1.0 + std::erf(s))) / (2.0 * beta * std::sqrt(kPi_h));
}

void build_plan(const hs_gas *g, const hs_case *cs, int n, Plan &P)
{
    P.gas.m = g->m;
    P.gas.R = kKB_h / g->m;
    P.gas.Pr = g->Pr;
    P.gas.gamma = g->gamma;
    P.gas.mu_ref = g->mu_ref;
    P.gas.T_ref = g->T_ref;
    P.gas.omega = g->omega;
    P.gas.K_vhs = vhs_K(g);
    P.gas.vhs_exp = 2.0 - 2.0 * g->omega;
    int64_t cell0 = 0;
    for (int i = 0; i < n; ++i) if (cs[i].dim == 0) P.any_0d = true;
    for (int i = 0; i < n; ++i) if (cs[i].mesh) P.any_mesh = true;
    for (int i = 0; i < n; ++i) if (cs[i].mesh && cs[i].dim == 2) P.any_quad = true;
    for (int i = 0; i < n; ++i) if (cs[i].mesh && cs[i].dim == 3) P.any_hex = true;
    for (int i = 0; i < n; ++i) {
        const hs_case &c = cs[i];
        CaseDev d;
        std::memset(&d, 0, sizeof(d));
        d.dim = c.dim;
        d.mesh = c.mesh ? 1 : 0;
        d.n[0] = c.mesh ? c.mesh->n_cells : c.nx;
        d.n[1] = c.dim >= 2 && !c.mesh ? c.ny : 1;
        d.n[2] = c.dim >= 3 && !c.mesh ? c.nz : 1;
        const int64_t nc = (int64_t)d.n[0] * d.n[1] * d.n[2];
        d.cell0 = (int32_t)cell0;
        d.ncells = (int32_t)nc;
        for (int a = 0; a < 6; ++a) d.bc[a] = c.bc[a];
        d.body = c.body;
        d.seed_lo = (uint32_t)(c.seed & 0xffffffffu);
        d.seed_hi = (uint32_t)(c.seed >> 32);
        d.n_steady = c.n_steady;
        d.capacity = c.capacity;
        d.surf0 = P.cases.empty() ? 0 : P.cases.back().surf0 + P.cases.back().n_surf;
        d.n_surf = c.n_surf;
        d.adapt_dt = c.adapt_dt;
        for (int a = 0; a < 3; ++a) {
            d.lo[a] = c.lo[a];
            d.h[a] = c.h[a];
            d.dt_over_h[a] = c.dt_G / c.h[a];
            d.body_c[a] = c.body_c[a];
            d.in_u[a] = c.inflow.u[a];
        }
        d.inv_n[0] = 1.0 / (double)std::max(d.n[0], 1);
        d.inv_n[1] = 1.0 / ((double)std::max(d.n[0], 1) * (double)std::max(d.n[1], 1));
        d.body_r = c.body_r;
        d.body_T = c.body_T;
        d.F_N = c.F_N;
        d.dt_G = c.dt_G;
        double L = c.h[0];
        for (int a = 1; a < c.dim; ++a) if (c.h[a] < L) L = c.h[a];
        d.L_cell = L;
        d.sigc0 = P.gas.K_vhs * std::pow(10.0 * std::sqrt(kKB_h * c.T_sigma / g->m), 2.0 - 2.0 * g->omega);
        d.in_n = c.inflow.n;
        d.in_T = c.inflow.T;
        for (int a = 0; a < 3; ++a) {
            d.bb_lo[a] = 0;
            d.bb_hi[a] = d.n[a] - 1;
        }
        if (c.body != HS_BODY_NONE && !c.mesh) {
            const int na = c.body == HS_BODY_SPHERE ? 3 : 2;
            for (int a = 0; a < na; ++a) {
                d.bb_lo[a] = (int32_t)std::floor((c.body_c[a] - c.body_r - c.lo[a]) / c.h[a]) - 1;
                d.bb_hi[a] = (int32_t)std::floor((c.body_c[a] + c.body_r - c.lo[a]) / c.h[a]) + 1;
            }
            P.any_body = true;
        }
        d.region0 = (int32_t)P.rstate.size();
        d.nregions = c.n_regions;
        for (int r = 0; r < c.n_regions; ++r) {
            for (int k = 0; k < 6; ++k) P.rbox.push_back(c.region_box ? c.region_box[6 * r + k] : 0.0);
            StateDev st;
            st.n = c.region_state[r].n;
            for (int a = 0; a < 3; ++a) st.u[a] = c.region_state[r].u[a];
            st.T = c.region_state[r].T;
            P.rstate.push_back(st);
        }
        if (P.any_0d) {
            const double tau0 = c.dim == 0 ? g->mu_ref * std::pow(c.region_state[0].T / g->T_ref, g->omega) /
                                                 (c.region_state[0].n * kKB_h * c.region_state[0].T)
                                           : 0.0;
            d.tau0 = tau0;
            for (int64_t k = 0; k < nc; ++k) P.dtcell.push_back(c.dim == 0 ? c.dt_over_tau[k] * tau0 : c.dt_G);
        }
        // inflow faces: sides -x,+x,-y,+y,-z,+z; boundary cells x-fastest; slot filter
        // (a mesh: its INFLOW edges, in cell and edge order)
        d.face0 = (int32_t)P.faces.size();
        if (P.any_mesh) P.mgeo.resize(2 * (size_t)(cell0 + nc), 0.0);
        if (P.any_hex) {
            const int32_t hnode0 = (int32_t)(P.hxyz.size() / 3);
            P.hnode.resize(8 * (size_t)(cell0 + nc), 0);
            P.hnbr.resize(8 * (size_t)(cell0 + nc), HS_EDGE_OUTFLOW);
            if (c.mesh && c.dim == 3) {
                const hs_mesh *m = c.mesh;
                P.hxyz.insert(P.hxyz.end(), m->xy, m->xy + 3 * (size_t)m->n_nodes);
                for (int64_t k = 0; k < nc; ++k) {
                    for (int j = 0; j < 8; ++j) P.hnode[8 * (cell0 + k) + j] = hnode0 + m->quad[8 * k + j];
                    for (int f = 0; f < 6; ++f) {
                        const int32_t nb = m->nbr[6 * k + f];
                        P.hnbr[8 * (cell0 + k) + f] = nb >= 0 ? (int32_t)(cell0 + nb) : nb;
                    }
                    double Ph[8][3], v, am;
                    hex_nodes_h(m, k, Ph);
                    hex_geometry_h(Ph, v, am);
                    P.mgeo[2 * (cell0 + k)] = v;
                    P.mgeo[2 * (cell0 + k) + 1] = v / am;      // volume over the largest face
                    for (int f = 0; f < 6; ++f) {
                        if (m->nbr[6 * k + f] != HS_EDGE_INFLOW) continue;
                        const double *A;
                        double nf[3];
                        hex_face_h(Ph, f, A, nf);
                        const double ln = std::sqrt(dot3h(nf, nf));
                        if (!(ln > 0.0)) continue;
                        const double nrm[3] = {-nf[0] / ln, -nf[1] / ln, -nf[2] / ln};
                        FaceDev fc;
                        fc.cell = (int32_t)(cell0 + k);
                        fc.side = f;
                        fc.case_id = i;
                        fc.local = (int32_t)(P.faces.size() - d.face0);
                        fc.lambda = edge_flux3(g, c.inflow, nrm) * (0.5 * ln) * c.dt_G / c.F_N;
                        P.faces.push_back(fc);
                    }
                }
            }
        }
        if (P.any_quad) {
            const int32_t node0 = (int32_t)(P.mxy.size() / 2);
            P.mquad.resize(4 * (size_t)(cell0 + nc), 0);
            P.mnbr.resize(4 * (size_t)(cell0 + nc), HS_EDGE_OUTFLOW);
            if (c.mesh && c.dim == 2) {
                const hs_mesh *m = c.mesh;
                P.mxy.insert(P.mxy.end(), m->xy, m->xy + 2 * (size_t)m->n_nodes);
                for (int64_t k = 0; k < nc; ++k) {
                    const int32_t *q = &m->quad[4 * k];
                    double Pq[4][2];
                    for (int j = 0; j < 4; ++j) {
                        P.mquad[4 * (cell0 + k) + j] = node0 + q[j];
                        const int32_t nb = m->nbr[4 * k + j];
                        P.mnbr[4 * (cell0 + k) + j] = nb >= 0 ? (int32_t)(cell0 + nb) : nb;
                        Pq[j][0] = m->xy[2 * q[j]];
                        Pq[j][1] = m->xy[2 * q[j] + 1];
                    }
                    // area from two triangles at node 0; L_cell = area / longest edge
                    const double area = 0.5 * (cross2(Pq[0], Pq[1], Pq[0], Pq[2]) + cross2(Pq[0], Pq[2], Pq[0], Pq[3]));
                    double lmax = 0.0;
                    for (int j = 0; j < 4; ++j) {
                        const double ex = Pq[(j + 1) & 3][0] - Pq[j][0], ey = Pq[(j + 1) & 3][1] - Pq[j][1];
                        const double l = std::sqrt(ex * ex + ey * ey);
                        if (l > lmax) lmax = l;
                    }
                    P.mgeo[2 * (cell0 + k)] = area * c.h[2];
                    P.mgeo[2 * (cell0 + k) + 1] = area / lmax;
                    for (int j = 0; j < 4; ++j) {
                        if (m->nbr[4 * k + j] != HS_EDGE_INFLOW) continue;
                        const double ex = Pq[(j + 1) & 3][0] - Pq[j][0], ey = Pq[(j + 1) & 3][1] - Pq[j][1];
                        const double len = std::sqrt(ex * ex + ey * ey);
                        const double nrm[2] = {-ey / len, ex / len};
                        FaceDev f;
                        f.cell = (int32_t)(cell0 + k);
                        f.side = j;
                        f.case_id = i;
                        f.local = (int32_t)(P.faces.size() - d.face0);
                        f.lambda = edge_flux(g, c.inflow, nrm) * (len * c.h[2]) * c.dt_G / c.F_N;
                        P.faces.push_back(f);
                    }
                }
            }
        }
        for (int s = 0; s < 2 * c.dim && !c.mesh; ++s) {
            if (c.bc[s] != HS_BC_INFLOW) continue;
            const int a = s / 2;
            const double sg = (s % 2 == 0) ? 1.0 : -1.0;
            double area = 1.0;
            for (int t = 0; t < 3; ++t) if (t != a) area *= c.h[t];
            const double lam = face_flux(g, c.inflow, a, sg) * area * c.dt_G / c.F_N;
            for (int64_t k = 0; k < nc; ++k) {
                const int ijk[3] = {(int)(k % d.n[0]), (int)((k / d.n[0]) % d.n[1]), (int)(k / ((int64_t)d.n[0] * d.n[1]))};
                if (ijk[a] != ((s % 2 == 0) ? 0 : d.n[a] - 1)) continue;
                bool ok = true;
                for (int t = 0; t < c.dim; ++t) {
                    if (t == a || !(c.slot_hi[t] > c.slot_lo[t])) continue;
                    const double ctr = c.lo[t] + ((double)ijk[t] + 0.5) * c.h[t];
                    if (!(ctr >= c.slot_lo[t] && ctr < c.slot_hi[t])) ok = false;
                }
                if (!ok) continue;
                FaceDev f;
                f.cell = (int32_t)(cell0 + k);
                f.side = s;
                f.case_id = i;
                f.local = (int32_t)(P.faces.size() - d.face0);
                f.lambda = lam;
                P.faces.push_back(f);
            }
        }
        d.nfaces = (int32_t)(P.faces.size() - d.face0);
        P.cases.push_back(d);
        cell0 += nc;
        P.capacity += c.capacity;
        P.dim_max = std::max(P.dim_max, c.dim);
        if (c.dim > 0) P.any_spatial = true;
    }
    P.ncells = cell0;
}

Layout make_layout(const Plan &P, hs_precision prec, uint32_t flags)
{
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
    const size_t es = prec == HS_FP64 ? 8 : 4;
    const size_t cap = (size_t)std::max<int64_t>(P.capacity, 1);
    const size_t nc = (size_t)P.ncells;
    // ---- the sim's data
    L.globals = take(sizeof(Globals));
    L.cases = take(sizeof(CaseDev) * P.cases.size());
    L.faces = take(sizeof(FaceDev) * std::max<size_t>(P.faces.size(), 1));
    L.rbox = take(sizeof(double) * std::max<size_t>(P.rbox.size(), 1));
    L.rstate = take(sizeof(StateDev) * std::max<size_t>(P.rstate.size(), 1));
    L.dtcell = P.any_0d ? take(sizeof(double) * nc) : 0;
    for (int b = 0; b < 2; ++b) {
        for (int a = 0; a < 3; ++a) L.pos[b][a] = a < P.dim_max ? take(es * cap) : 0;
        for (int a = 0; a < 3; ++a) L.vel[b][a] = take(es * cap);
        L.cell[b] = take(4 * cap);
        L.id[b] = take(4 * cap);
    }
    L.sigc = take(8 * nc);
    L.acc = take(8 * 13 * nc);
    L.vol = take(8 * nc);
    size_t nsurf = 0;
    for (const auto &c : P.cases) nsurf += (size_t)c.n_surf;
    L.surf_bytes = 8 * 7 * (size_t)kSurfCopies * std::max<size_t>(nsurf, 1);
    L.surf = take(L.surf_bytes);
    L.trace = (flags & HS_FLAG_TRACE) ? take(sizeof(TraceDev) * nc) : 0;
    if (P.any_mesh) L.mgeo = take(sizeof(double) * 2 * nc);
    if (P.any_quad) {
        L.mxy = take(sizeof(double) * std::max<size_t>(P.mxy.size(), 2));
        L.mquad = take(sizeof(int32_t) * 4 * nc);
        L.mnbr = take(sizeof(int32_t) * 4 * nc);
    }
    if (P.any_hex) {
        L.hxyz = take(sizeof(double) * std::max<size_t>(P.hxyz.size(), 3));
        L.hnode = take(sizeof(int32_t) * 8 * nc);
        L.hnbr = take(sizeof(int32_t) * 8 * nc);
    }
    // ---- scratch of the step
    L.scratch_begin = o;
    // new cells and slots of the move; the block-per-cell kernel also uses them as scratch
    // (claim words, sorted sources) for cells too dense for LDS, so every batch has them
    L.newcell = take(4 * cap);
    L.slot = take(4 * cap);
    L.perm = P.any_spatial ? take(4 * cap) : 0;
    L.work = P.any_body ? take(4 * cap) : 0;
    L.count = take(4 * nc);
    L.cstart = take(4 * (nc + 1));
    L.facecnt = take(4 * std::max<size_t>(P.faces.size(), 1));
    L.facestart = take(4 * (P.faces.size() + 1));
    L.scanpart = take(4 * (nc / (kBlock * 16) + 2));
    L.big = take(4 * std::max<size_t>(nc, dense_list_length(P.capacity, nc, kDenseClasses)));
    L.tiles = take(4 * ((cap + 4 * nc) / tile_width() + P.cases.size() + 3));
    L.tilecase = take(4 * ((cap + 4 * nc) / tile_width() + P.cases.size() + 3));
    L.cellrec = take(8 * 16 * nc);
    size_t maxcase = 1;
    for (const auto &c : P.cases) maxcase = std::max<size_t>(maxcase, (size_t)c.ncells);
    size_t maxsurf = 0;
    for (const auto &c : P.cases) maxsurf = std::max<size_t>(maxsurf, (size_t)c.n_surf);
    L.out = take(8 * std::max<size_t>(8 * maxcase, 8 * maxsurf + 5));
    L.total = o;
    return L;
}

}  // namespace

struct hs_sim {
    hs_precision prec;
    uint32_t flags;
    hipStream_t stream;
    // second stream of the step: the dense-cell kernel runs on it beside the scalar and tile
    // kernels, forked from and joined back into `stream` by the two events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    char *ws;                            // the sim's data (the caller's workspace)
    char *scratch;                       // the step's scratch arrays
    size_t ws_bytes;
    Plan plan;
    Layout lay;
    Ctx ctx;
    std::vector<hs_case> cases;
    int failed = 0;
    std::string err;
    bool graph_ready = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    uint32_t timing = 0;                 // mask of timed kernel groups
    int timing_period = 1;               // timed: every timing_period-th step of hs_step
    struct StepEvents {
        hipEvent_t b[HS_NUM_KERNELS], e[HS_NUM_KERNELS];
    };
    std::vector<StepEvents> events;      // one record per timed step
    int64_t timed_steps = 0;
};

namespace {

// Device address of the layout offset `off` (data part or scratch part).
char *at(const hs_sim *s, size_t off)
{
    return off < s->lay.scratch_begin ? s->ws + off : s->scratch + (off - s->lay.scratch_begin);
}

hs_status fail(hs_sim *s, hs_status st, const std::string &why)
{
    if (s) {
        s->err = why;
        if (st != HS_ERR_ARG) s->failed = st;
    }
    return st;
}

#define HIPCHK(sim, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return fail(sim, HS_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

hs_status read_globals(hs_sim *s, Globals &G)
{
    HIPCHK(s, hipStreamSynchronize(s->stream));
    HIPCHK(s, hipMemcpy(&G, at(s, s->lay.globals), sizeof(Globals), hipMemcpyDeviceToHost));
    return HS_OK;
}

hs_status check_device(hs_sim *s)
{
    if (s->failed) return HS_ERR_STATE;
    Globals G;
    hs_status st = read_globals(s, G);
    if (st) return st;
    if (G.err) {
        std::string why = "device error:";
        hs_status code = HS_ERR_STATE;
        if (G.err & kErrCapacity) { why += " particle capacity exceeded"; code = HS_ERR_CAPACITY; }
        if (G.err & kErrNumeric) { why += " non-finite moment"; if (code == HS_ERR_STATE) code = HS_ERR_NUMERIC; }
        if (G.err & kErrState) { why += " inconsistent state"; }
        s->err = why;
        s->failed = code;
        return code;
    }
    return HS_OK;
}

void enqueue_step(hs_sim *s, int timed)
{
    const Ctx &c = s->ctx;
    void *st = (void *)s->stream;
    hs_sim::StepEvents *ev = nullptr;
    if (timed) {
        s->events.emplace_back();
        ev = &s->events.back();
        for (int k = 0; k < HS_NUM_KERNELS; ++k) ev->b[k] = ev->e[k] = nullptr;
    }
    auto mark = [&](int k, bool begin, hipStream_t on) {
        if (!ev || !((s->timing >> k) & 1u)) return;
        hipEvent_t &e = begin ? ev->b[k] : ev->e[k];
        if (hipEventCreate(&e) != hipSuccess) { e = nullptr; return; }
        (void)hipEventRecord(e, on);
    };
    const hipStream_t ms = s->stream;
    mark(HS_KERNEL_STEP, true, ms);
    if (s->plan.any_spatial) {
        mark(HS_KERNEL_INJECT, true, ms);
        Launch::inject(c, st);
        mark(HS_KERNEL_INJECT, false, ms);
        mark(HS_KERNEL_MOVE, true, ms);
        Launch::move_count(c, st, s->plan.any_body ? 1 : 0);
        mark(HS_KERNEL_MOVE, false, ms);
        mark(HS_KERNEL_SCAN, true, ms);
        Launch::scan_cells(c, st, 1);
        mark(HS_KERNEL_SCAN, false, ms);
        mark(HS_KERNEL_SCATTER, true, ms);
        Launch::scatter(c, st);
        mark(HS_KERNEL_SCATTER, false, ms);
    }
    // cells denser than the tile limit: their kernel sorts, gathers and collides its cells
    // alone (from the scatter's permutation), sharing no cell with the gather, scalar and
    // tile kernels, so it runs on the side stream while they run
    // (a sim without a side stream runs it first on its own stream)
    const hipStream_t ds = s->side ? s->side : ms;
    if (s->side) {
        (void)hipEventRecord(s->ev_fork, ms);
        (void)hipStreamWaitEvent(s->side, s->ev_fork, 0);
    }
    mark(HS_KERNEL_DENSE, true, ds);
    Launch::dense(c, (void *)ds);
    mark(HS_KERNEL_DENSE, false, ds);
    if (s->side) (void)hipEventRecord(s->ev_join, s->side);
    mark(HS_KERNEL_GATHER, true, ms);
    Launch::gather(c, st);
    mark(HS_KERNEL_GATHER, false, ms);
    mark(HS_KERNEL_SCALARS, true, ms);
    Launch::scalars(c, st);
    mark(HS_KERNEL_SCALARS, false, ms);
    mark(HS_KERNEL_COLLIDE, true, ms);
    Launch::collide(c, st);
    mark(HS_KERNEL_COLLIDE, false, ms);
    if (s->side) (void)hipStreamWaitEvent(ms, s->ev_join, 0);
    Launch::finish_step(c, st);
    mark(HS_KERNEL_STEP, false, ms);
}

}  // namespace

extern "C" {

hs_status hs_plan(const hs_gas *gas, const hs_case *cases, int n_cases, hs_precision prec, uint32_t flags,
                  size_t *dev_bytes)
{
    std::string why;
    if (!dev_bytes || (prec != HS_FP64 && prec != HS_FP32_MIXED)) return HS_ERR_ARG;
    hs_status st = validate(gas, cases, n_cases, why);
    if (st) return st;
    Plan P;
    build_plan(gas, cases, n_cases, P);
    const Layout L = make_layout(P, prec, flags & ~(uint32_t)HS_FLAG_STATIC_SCRATCH);
    if (flags & HS_FLAG_STATIC_SCRATCH) {
        // the caller's part only; the scratch part must fit the library's fixed array
        if (L.total - L.scratch_begin > (size_t)HS_STATIC_SCRATCH_BYTES) return HS_ERR_CAPACITY;
        *dev_bytes = L.scratch_begin;
    } else {
        *dev_bytes = L.total;
    }
    return HS_OK;
}

}  // extern "C"

namespace {

// Shared set-up of hs_init_particles and hs_init_particles_static: `data` holds the sim's
// data part of the layout (>= scratch_begin bytes, or the whole layout when `scratch` is
// null), `scratch` the scratch part; `side_stream`: fork the dense-cell kernel onto a second
// stream (else it runs on the caller's stream).
hs_status create_sim(const hs_gas *gas, const hs_case *cases, int n_cases, hs_precision prec, uint32_t flags,
                     char *data, size_t data_bytes, char *scratch, size_t scratch_bytes, void *hip_stream,
                     bool side_stream, hs_sim **out)
{
    std::string why;
    if (!out || !data || (prec != HS_FP64 && prec != HS_FP32_MIXED)) return HS_ERR_ARG;
    hs_status st = validate(gas, cases, n_cases, why);
    if (st) return st;
    hs_sim *s = new hs_sim();
    s->prec = prec;
    s->flags = flags;
    s->stream = (hipStream_t)hip_stream;
    s->ws = data;
    s->ws_bytes = data_bytes;
    build_plan(gas, cases, n_cases, s->plan);
    s->lay = make_layout(s->plan, prec, flags);
    s->scratch = scratch ? scratch : data + s->lay.scratch_begin;
    const size_t need_data = scratch ? s->lay.scratch_begin : s->lay.total;
    const size_t need_scratch = s->lay.total - s->lay.scratch_begin;
    if (data_bytes < need_data || (scratch && scratch_bytes < need_scratch)) {
        delete s;
        return scratch && scratch_bytes < need_scratch ? HS_ERR_CAPACITY : HS_ERR_ARG;
    }
    s->cases.assign(cases, cases + n_cases);
    const Layout &L = s->lay;
    Ctx &c = s->ctx;
    std::memset(&c, 0, sizeof(c));
    c.cases = (const CaseDev *)at(s, L.cases);
    c.faces = (const FaceDev *)at(s, L.faces);
    c.region_box = (const double *)at(s, L.rbox);
    c.region_state = (const StateDev *)at(s, L.rstate);
    c.dt_cell = s->plan.any_0d ? (const double *)at(s, L.dtcell) : nullptr;
    c.gas = s->plan.gas;
    for (int b = 0; b < 2; ++b) {
        for (int a = 0; a < 3; ++a) {
            c.buf[b].pos[a] = a < s->plan.dim_max ? (void *)at(s, L.pos[b][a]) : nullptr;
            c.buf[b].vel[a] = at(s, L.vel[b][a]);
        }
        c.buf[b].cell = (int32_t *)at(s, L.cell[b]);
        c.buf[b].id = (uint32_t *)at(s, L.id[b]);
    }
    c.newcell = (int32_t *)at(s, L.newcell);
    c.slot = (int32_t *)at(s, L.slot);
    c.perm = s->plan.any_spatial ? (int32_t *)at(s, L.perm) : nullptr;
    c.count = (int32_t *)at(s, L.count);
    c.cstart = (int32_t *)at(s, L.cstart);
    c.sigc = (double *)at(s, L.sigc);
    c.acc = (double *)at(s, L.acc);
    c.vol = (double *)at(s, L.vol);
    c.face_cnt = (int32_t *)at(s, L.facecnt);
    c.face_start = (int32_t *)at(s, L.facestart);
    c.scan_part = (int32_t *)at(s, L.scanpart);
    c.big_list = (int32_t *)at(s, L.big);
    for (int k = 0; k <= kDenseClasses; ++k)
        c.big_off[k] = (int32_t)dense_list_length(s->plan.capacity, s->plan.ncells, k);
    c.tile_cell = (int32_t *)at(s, L.tiles);
    c.tile_case = (int32_t *)at(s, L.tilecase);
    c.cellrec = (double *)at(s, L.cellrec);
    c.surf = (double *)at(s, L.surf);
    {
        size_t ns = 0;
        for (const auto &cd : s->plan.cases) ns += (size_t)cd.n_surf;
        c.n_surf_total = (int32_t)ns;
    }
    c.work = s->plan.any_body ? (int32_t *)at(s, L.work) : nullptr;
    if (s->plan.any_mesh) c.mgeo = (const double *)at(s, L.mgeo);
    if (s->plan.any_quad) {
        c.mxy = (const double *)at(s, L.mxy);
        c.mquad = (const int32_t *)at(s, L.mquad);
        c.mnbr = (const int32_t *)at(s, L.mnbr);
    }
    if (s->plan.any_hex) {
        c.hxyz = (const double *)at(s, L.hxyz);
        c.hnode = (const int32_t *)at(s, L.hnode);
        c.hnbr = (const int32_t *)at(s, L.hnbr);
    }
    c.tile_w = tile_width();
    c.dim_max = s->plan.dim_max;
    c.trace = (flags & HS_FLAG_TRACE) ? (TraceDev *)at(s, L.trace) : nullptr;
    c.g = (Globals *)at(s, L.globals);
    c.n_cases = n_cases;
    c.n_faces = (int32_t)s->plan.faces.size();
    c.ncells_total = (int32_t)s->plan.ncells;
    c.cap_wave = cap_wave();
    c.cap_block = cap_block(prec);
    c.precision = prec;
    c.capacity = s->plan.capacity;

    auto up = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(at(s, off), src, bytes, hipMemcpyHostToDevice, s->stream);
    };
    hipError_t e = hipSuccess;
    e = e ? e : up(L.cases, s->plan.cases.data(), sizeof(CaseDev) * s->plan.cases.size());
    e = e ? e : up(L.faces, s->plan.faces.data(), sizeof(FaceDev) * s->plan.faces.size());
    e = e ? e : up(L.rbox, s->plan.rbox.data(), sizeof(double) * s->plan.rbox.size());
    e = e ? e : up(L.rstate, s->plan.rstate.data(), sizeof(StateDev) * s->plan.rstate.size());
    if (s->plan.any_0d) e = e ? e : up(L.dtcell, s->plan.dtcell.data(), sizeof(double) * s->plan.dtcell.size());
    if (s->plan.any_mesh) e = e ? e : up(L.mgeo, s->plan.mgeo.data(), sizeof(double) * s->plan.mgeo.size());
    if (s->plan.any_quad) {
        e = e ? e : up(L.mxy, s->plan.mxy.data(), sizeof(double) * s->plan.mxy.size());
        e = e ? e : up(L.mquad, s->plan.mquad.data(), sizeof(int32_t) * s->plan.mquad.size());
        e = e ? e : up(L.mnbr, s->plan.mnbr.data(), sizeof(int32_t) * s->plan.mnbr.size());
    }
    if (s->plan.any_hex) {
        e = e ? e : up(L.hxyz, s->plan.hxyz.data(), sizeof(double) * s->plan.hxyz.size());
        e = e ? e : up(L.hnode, s->plan.hnode.data(), sizeof(int32_t) * s->plan.hnode.size());
        e = e ? e : up(L.hnbr, s->plan.hnbr.data(), sizeof(int32_t) * s->plan.hnbr.size());
    }
    e = e ? e : hipMemsetAsync(at(s, L.globals), 0, sizeof(Globals), s->stream);
    e = e ? e : hipMemsetAsync(at(s, L.surf), 0, L.surf_bytes, s->stream);
    if (e != hipSuccess) {
        std::string m = hipGetErrorString(e);
        delete s;
        (void)m;
        return HS_ERR_DEVICE;
    }
    const int fill = (flags & HS_FLAG_NO_PARTICLES) ? 0 : 1;
    Ctx ci = c;
    if (fill) Launch::init_cells(ci, s->stream);
    else Launch::init_count(ci, s->stream);
    Launch::scan_cells(ci, s->stream, 0);
    if (fill) Launch::init_fill(ci, s->stream);
    Launch::init_finish(ci, s->stream);
    if (!s->plan.any_spatial) launch_build_big(ci, s->stream);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (side_stream) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
        if (s->side) (void)hipStreamDestroy(s->side);
        delete s;
        return HS_ERR_DEVICE;
    }
    *out = s;
    hs_status cs = check_device(s);
    return cs;
}

}  // namespace

extern "C" {

hs_status hs_init_particles(const hs_gas *gas, const hs_case *cases, int n_cases, hs_precision prec,
                            uint32_t flags, void *dev_workspace, size_t dev_bytes, void *hip_stream, hs_sim **out)
{
    if (flags & HS_FLAG_STATIC_SCRATCH) return HS_ERR_ARG;
    return create_sim(gas, cases, n_cases, prec, flags, (char *)dev_workspace, dev_bytes, nullptr, 0, hip_stream,
                      true, out);
}

hs_status hs_init_particles_static(const hs_gas *gas, const hs_case *cases, int n_cases, hs_precision prec,
                                   uint32_t flags, void *dev_data, size_t data_bytes, void *hip_stream,
                                   hs_sim **out)
{
    if (!out || !dev_data) return HS_ERR_ARG;
    *out = nullptr;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    if (static_scratch(&scratch, &scratch_bytes) != 0) return HS_ERR_DEVICE;
    return create_sim(gas, cases, n_cases, prec, flags & ~(uint32_t)HS_FLAG_STATIC_SCRATCH, (char *)dev_data,
                      data_bytes, (char *)scratch, scratch_bytes, hip_stream, false, out);
}

hs_status hs_step(hs_sim *s, int64_t n)
{
    if (!s || n < 0) return HS_ERR_ARG;
    if (s->failed) return HS_ERR_STATE;
    if (s->timing) {
        for (int64_t k = 0; k < n; ++k) enqueue_step(s, (s->timed_steps + k) % s->timing_period == 0 ? 1 : 0);
        s->timed_steps += n;
    } else if (s->flags & HS_FLAG_GRAPH) {
        if (!s->graph_ready) {
            HIPCHK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
            enqueue_step(s, 0);
            HIPCHK(s, hipStreamEndCapture(s->stream, &s->graph));
            HIPCHK(s, hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0));
            s->graph_ready = true;
        }
        for (int64_t k = 0; k < n; ++k) HIPCHK(s, hipGraphLaunch(s->gexec, s->stream));
    } else {
        for (int64_t k = 0; k < n; ++k) enqueue_step(s, 0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(s, HS_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    return HS_OK;
}

hs_status hs_surface_sums(hs_sim *s, int c, double *sums7)
{
    if (!s || !sums7 || c < 0 || c >= (int)s->plan.cases.size() || s->plan.cases[c].n_surf <= 0) return HS_ERR_ARG;
    hs_status st = check_device(s);
    if (st) return st;
    const CaseDev &cs = s->plan.cases[c];
    double *out = (double *)at(s, s->lay.out);
    launch_surface_reduce(s->ctx, s->stream, c, out);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(sums7, out, 8 * 7 * (size_t)cs.n_surf, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return HS_OK;
}

hs_status hs_surface_sample(hs_sim *s, int c, double *elem8, double *body5, int64_t *n_samples)
{
    if (!s || !elem8 || !body5 || c < 0 || c >= (int)s->plan.cases.size() || s->plan.cases[c].n_surf <= 0)
        return HS_ERR_ARG;
    hs_status st = check_device(s);
    if (st) return st;
    const int ns = s->plan.cases[c].n_surf;
    double *out = (double *)at(s, s->lay.out);
    launch_surface_finalize(s->ctx, s->stream, c, out);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(elem8, out, 8 * 8 * (size_t)ns, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(body5, out + 8 * (size_t)ns, 8 * 5, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (n_samples) {
        Globals G;
        st = read_globals(s, G);
        if (st) return st;
        *n_samples = G.n_samples[c];
    }
    return HS_OK;
}

hs_status hs_step_dt(hs_sim *s, int c, double *dt_next, double *t_sampled)
{
    if (!s || c < 0 || c >= (int)s->plan.cases.size()) return HS_ERR_ARG;
    hs_status st = check_device(s);
    if (st) return st;
    Globals G;
    if ((st = read_globals(s, G))) return st;
    if (dt_next) *dt_next = G.dt_cur[c];
    if (t_sampled) *t_sampled = G.t_sampled[c];
    return HS_OK;
}

hs_status hs_dsmc_ratio(hs_sim *s, int c, double *ratio)
{
    if (!s || !ratio || c < 0 || c >= (int)s->plan.cases.size()) return HS_ERR_ARG;
    hs_status st = check_device(s);
    if (st) return st;
    const int nc = s->plan.cases[c].ncells;
    double *out = (double *)at(s, s->lay.out);
    launch_dsmc_ratio(s->ctx, s->stream, c, nc, out);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(ratio, out, 8 * (size_t)nc, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return HS_OK;
}

hs_status hs_sync(hs_sim *s)
{
    if (!s) return HS_ERR_ARG;
    return check_device(s);
}

int64_t hs_num_cells(const hs_sim *s, int c)
{
    if (!s || c < 0 || c >= (int)s->plan.cases.size()) return -1;
    return s->plan.cases[c].ncells;
}

static hs_status case_range(hs_sim *s, int c, int32_t &a, int32_t &b)
{
    const CaseDev &cs = s->plan.cases[c];
    HIPCHK(s, hipMemcpy(&a, s->ctx.cstart + cs.cell0, 4, hipMemcpyDeviceToHost));
    HIPCHK(s, hipMemcpy(&b, s->ctx.cstart + cs.cell0 + cs.ncells, 4, hipMemcpyDeviceToHost));
    return HS_OK;
}

int64_t hs_num_particles(hs_sim *s, int c)
{
    if (!s || c < 0 || c >= (int)s->plan.cases.size()) return -1;
    if (check_device(s)) return -1;
    int32_t a, b;
    if (case_range(s, c, a, b)) return -1;
    return (int64_t)b - a;
}

hs_status hs_sample_moments(hs_sim *s, int c, int mode, double *n, double *u3, double *T, double *q3,
                            int64_t *n_samples)
{
    if (!s || c < 0 || c >= (int)s->plan.cases.size() || (mode != 0 && mode != 1)) return HS_ERR_ARG;
    hs_status st = check_device(s);
    if (st) return st;
    const int nc = s->plan.cases[c].ncells;
    double *out = (double *)at(s, s->lay.out);
    if (mode == 0) launch_finalize(s->ctx, s->stream, c, nc, out);
    else launch_moments_now(s->ctx, s->stream, c, nc, out);
    std::vector<double> h((size_t)nc * 8);
    HIPCHK(s, hipMemcpyAsync(h.data(), out, h.size() * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int k = 0; k < nc; ++k) {
        const double *o = &h[8 * (size_t)k];
        if (n) n[k] = o[0];
        if (T) T[k] = o[4];
        for (int a = 0; a < 3; ++a) {
            if (u3) u3[3 * k + a] = o[1 + a];
            if (q3) q3[3 * k + a] = o[5 + a];
        }
    }
    if (n_samples) {
        Globals G;
        st = read_globals(s, G);
        if (st) return st;
        *n_samples = G.n_samples[c];
    }
    return HS_OK;
}

size_t hs_state_bytes(hs_sim *s, int c)
{
    if (!s || c < 0 || c >= (int)s->plan.cases.size()) return 0;
    if (check_device(s)) return 0;
    int32_t a, b;
    if (case_range(s, c, a, b)) return 0;
    const size_t np = (size_t)(b - a), nc = (size_t)s->plan.cases[c].ncells;
    const size_t es = s->prec == HS_FP64 ? 8 : 4;
    return sizeof(hs_state_header) + np * (6 * es + 4 + 8) + nc * 8 * 14;
}

hs_status hs_export_state(hs_sim *s, int c, void *host_buf, size_t bytes)
{
    if (!s || !host_buf || c < 0 || c >= (int)s->plan.cases.size()) return HS_ERR_ARG;
    hs_status st = check_device(s);
    if (st) return st;
    const size_t need = hs_state_bytes(s, c);
    if (bytes < need) return HS_ERR_ARG;
    int32_t a, b;
    if ((st = case_range(s, c, a, b))) return st;
    Globals G;
    if ((st = read_globals(s, G))) return st;
    const CaseDev &cs = s->plan.cases[c];
    const size_t np = (size_t)(b - a), nc = (size_t)cs.ncells;
    const size_t es = s->prec == HS_FP64 ? 8 : 4;
    hs_state_header hd;
    hd.magic = kMagic;
    hd.version = 2;
    hd.precision = s->prec;
    hd.dim = cs.dim;
    hd.np = (int64_t)np;
    hd.ncells = (int64_t)nc;
    hd.next_id = G.next_id[c];
    hd.step = G.step;
    hd.n_samples = G.n_samples[c];
    hd.dt_next = G.dt_cur[c];
    hd.t_sampled = G.t_sampled[c];
    char *p = (char *)host_buf;
    std::memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    const PartBuf &B = s->ctx.buf[G.step & 1];
    for (int d = 0; d < 3; ++d) {
        if (d < cs.dim && np) HIPCHK(s, hipMemcpy(p, (char *)B.pos[d] + es * a, es * np, hipMemcpyDeviceToHost));
        else std::memset(p, 0, es * np);
        p += es * np;
    }
    for (int d = 0; d < 3; ++d) {
        if (np) HIPCHK(s, hipMemcpy(p, (char *)B.vel[d] + es * a, es * np, hipMemcpyDeviceToHost));
        p += es * np;
    }
    int32_t *cellp = (int32_t *)p;
    if (np) HIPCHK(s, hipMemcpy(p, B.cell + a, 4 * np, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < np; ++i) cellp[i] -= cs.cell0;
    p += 4 * np;
    {
        // ids are kept as their low 32 bits (full_id)
        std::vector<uint32_t> low(np);
        if (np) HIPCHK(s, hipMemcpy(low.data(), B.id + a, 4 * np, hipMemcpyDeviceToHost));
        int64_t *idp = (int64_t *)p;
        for (size_t i = 0; i < np; ++i) idp[i] = full_id(low[i], hd.next_id);
    }
    p += 8 * np;
    HIPCHK(s, hipMemcpy(p, s->ctx.sigc + cs.cell0, 8 * nc, hipMemcpyDeviceToHost));
    p += 8 * nc;
    HIPCHK(s, hipMemcpy(p, s->ctx.acc + 13 * (size_t)cs.cell0, 8 * 13 * nc, hipMemcpyDeviceToHost));
    return HS_OK;
}

hs_status hs_import_state(hs_sim *s, int c, const void *host_buf, size_t bytes)
{
    if (!s || !host_buf || c < 0 || c >= (int)s->plan.cases.size()) return HS_ERR_ARG;
    hs_status st = check_device(s);
    if (st) return st;
    if (bytes < sizeof(hs_state_header)) return HS_ERR_ARG;
    hs_state_header hd;
    std::memcpy(&hd, host_buf, sizeof(hd));
    const CaseDev &cs = s->plan.cases[c];
    const size_t es = s->prec == HS_FP64 ? 8 : 4;
    if (hd.magic != kMagic || hd.version != 2 || hd.precision != (uint32_t)s->prec || hd.dim != (uint32_t)cs.dim ||
        hd.ncells != cs.ncells || hd.np < 0 || hd.step < 0 || !(hd.t_sampled >= 0.0) ||
        (cs.dim > 0 ? !(hd.dt_next > 0.0) : !(hd.dt_next >= 0.0))) {
        s->err = "state header does not match the case";
        return HS_ERR_ARG;
    }
    const size_t np = (size_t)hd.np, nc = (size_t)cs.ncells;
    if (bytes < sizeof(hd) + np * (6 * es + 12) + nc * 8 * 14) return HS_ERR_ARG;
    if ((int64_t)np > cs.capacity) { s->err = "import exceeds the case capacity"; return HS_ERR_CAPACITY; }
    const char *p = (const char *)host_buf + sizeof(hd);
    const char *pos = p, *vel = p + 3 * es * np;
    const int32_t *cell = (const int32_t *)(p + 6 * es * np);
    const int64_t *ids = (const int64_t *)(p + 6 * es * np + 4 * np);
    const double *sigc = (const double *)(p + 6 * es * np + 12 * np);
    const double *acc = sigc + nc;
    auto rd = [&](const char *base, size_t i) -> double {
        return es == 8 ? ((const double *)base)[i] : (double)((const float *)base)[i];
    };
    for (size_t i = 0; i < np; ++i) {
        if (cell[i] < 0 || cell[i] >= cs.ncells || (i && cell[i] < cell[i - 1])) {
            s->err = "imported cells must be in range and non-decreasing";
            return HS_ERR_ARG;
        }
        // the state keeps ids as their low 32 bits: every id must be one of the case's last
        // 2^32 ids below its next id
        if (ids[i] < 0 || ids[i] >= hd.next_id || hd.next_id - ids[i] >= (int64_t)1 << 32) {
            s->err = "imported ids must lie in [next_id - 2^32 + 1, next_id)";
            return HS_ERR_ARG;
        }
        for (int d = 0; d < 3; ++d) {
            if (!std::isfinite(rd(vel + d * es * np, i))) { s->err = "non-finite imported velocity"; return HS_ERR_NUMERIC; }
            if (d < cs.dim) {
                const double x = rd(pos + d * es * np, i);
                if (cs.mesh ? !std::isfinite(x) : !(x >= 0.0 && x < 1.0)) {
                    s->err = "imported positions must be cell-relative in [0,1) (finite on a mesh)";
                    return HS_ERR_ARG;
                }
            }
        }
    }
    // rebuild the whole particle array with this case replaced
    Globals G;
    if ((st = read_globals(s, G))) return st;
    const int ncase = (int)s->plan.cases.size();
    std::vector<int32_t> cst((size_t)s->plan.ncells + 1);
    HIPCHK(s, hipMemcpy(cst.data(), s->ctx.cstart, 4 * cst.size(), hipMemcpyDeviceToHost));
    const PartBuf &Bo = s->ctx.buf[G.step & 1];
    const PartBuf &Bn = s->ctx.buf[hd.step & 1];
    const int dmax = s->plan.dim_max;
    std::vector<std::vector<char>> arrs(6);
    std::vector<int32_t> ncell;
    std::vector<uint32_t> nid;                 // ids as stored: their low 32 bits
    for (int k = 0; k < ncase; ++k) {
        const CaseDev &ck = s->plan.cases[k];
        if (k == c) {
            for (int d = 0; d < 3; ++d) {
                if (d < dmax) {
                    const size_t at = arrs[d].size();
                    arrs[d].resize(at + es * np);
                    std::memcpy(arrs[d].data() + at, pos + d * es * np, es * np);
                }
                const size_t at = arrs[3 + d].size();
                arrs[3 + d].resize(at + es * np);
                std::memcpy(arrs[3 + d].data() + at, vel + d * es * np, es * np);
            }
            for (size_t i = 0; i < np; ++i) {
                ncell.push_back(cell[i] + ck.cell0);
                nid.push_back((uint32_t)ids[i]);
            }
        } else {
            const int32_t a = cst[ck.cell0], b = cst[ck.cell0 + ck.ncells];
            const size_t m = (size_t)(b - a);
            for (int d = 0; d < 3; ++d) {
                if (d < dmax) {
                    const size_t at = arrs[d].size();
                    arrs[d].resize(at + es * m);
                    if (m) HIPCHK(s, hipMemcpy(arrs[d].data() + at, (char *)Bo.pos[d] + es * a, es * m, hipMemcpyDeviceToHost));
                }
                const size_t at = arrs[3 + d].size();
                arrs[3 + d].resize(at + es * m);
                if (m) HIPCHK(s, hipMemcpy(arrs[3 + d].data() + at, (char *)Bo.vel[d] + es * a, es * m, hipMemcpyDeviceToHost));
            }
            const size_t at = ncell.size();
            ncell.resize(at + m);
            nid.resize(at + m);
            if (m) {
                HIPCHK(s, hipMemcpy(ncell.data() + at, Bo.cell + a, 4 * m, hipMemcpyDeviceToHost));
                HIPCHK(s, hipMemcpy(nid.data() + at, Bo.id + a, 4 * m, hipMemcpyDeviceToHost));
            }
        }
    }
    const size_t total = ncell.size();
    if ((int64_t)total > s->plan.capacity) return HS_ERR_CAPACITY;
    for (int d = 0; d < 3; ++d) {
        if (d < dmax && total) HIPCHK(s, hipMemcpy(Bn.pos[d], arrs[d].data(), es * total, hipMemcpyHostToDevice));
        if (total) HIPCHK(s, hipMemcpy(Bn.vel[d], arrs[3 + d].data(), es * total, hipMemcpyHostToDevice));
    }
    if (total) {
        HIPCHK(s, hipMemcpy(Bn.cell, ncell.data(), 4 * total, hipMemcpyHostToDevice));
        HIPCHK(s, hipMemcpy(Bn.id, nid.data(), 4 * total, hipMemcpyHostToDevice));
    }
    std::vector<int32_t> cnt((size_t)s->plan.ncells + 1, 0);
    for (size_t i = 0; i < total; ++i) cnt[(size_t)ncell[i] + 1]++;
    for (size_t g = 1; g < cnt.size(); ++g) cnt[g] += cnt[g - 1];
    HIPCHK(s, hipMemcpy(s->ctx.cstart, cnt.data(), 4 * cnt.size(), hipMemcpyHostToDevice));
    HIPCHK(s, hipMemcpy(s->ctx.sigc + cs.cell0, sigc, 8 * nc, hipMemcpyHostToDevice));
    HIPCHK(s, hipMemcpy(s->ctx.acc + 13 * (size_t)cs.cell0, acc, 8 * 13 * nc, hipMemcpyHostToDevice));
    G.step = hd.step;
    G.n_live = (int32_t)total;
    G.n_total = (int32_t)total;
    G.n_new = (int32_t)total;
    for (int k = 0; k < kDenseClasses; ++k) G.n_big[k] = 0;
    G.n_work = 0;
    G.n_tiles = (int32_t)(((int64_t)total + 4 * s->plan.ncells + tile_width() - 1) / tile_width());
    G.next_id[c] = hd.next_id;
    G.n_samples[c] = hd.n_samples;
    G.dt_cur[c] = hd.dt_next;
    G.dt_next[c] = kInfBits;
    G.t_sampled[c] = hd.t_sampled;
    HIPCHK(s, hipMemcpy(at(s, s->lay.globals), &G, sizeof(G), hipMemcpyHostToDevice));
    Launch::tile_table(s->ctx, s->stream);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (!s->plan.any_spatial) {
        launch_build_big(s->ctx, s->stream);
        HIPCHK(s, hipGetLastError());
        HIPCHK(s, hipStreamSynchronize(s->stream));
    }
    return HS_OK;
}

hs_status hs_last_trace(hs_sim *s, int c, hs_trace *out)
{
    if (!s || !out || c < 0 || c >= (int)s->plan.cases.size() || !s->ctx.trace) return HS_ERR_ARG;
    hs_status st = check_device(s);
    if (st) return st;
    const CaseDev &cs = s->plan.cases[c];
    HIPCHK(s, hipMemcpy(out, s->ctx.trace + cs.cell0, sizeof(hs_trace) * cs.ncells, hipMemcpyDeviceToHost));
    return HS_OK;
}

hs_status hs_counters(hs_sim *s, int c, int64_t *out)
{
    if (!s || !out || c < 0 || c >= (int)s->plan.cases.size()) return HS_ERR_ARG;
    hs_status st = check_device(s);
    if (st) return st;
    Globals G;
    if ((st = read_globals(s, G))) return st;
    for (int k = 0; k < HS_NUM_COUNTERS; ++k) out[k] = G.counters[c][k];
    return HS_OK;
}

hs_status hs_set_timing(hs_sim *s, uint32_t mask)
{
    if (!s || (mask >> HS_NUM_KERNELS) != 0) return HS_ERR_ARG;
    s->timing = mask;
    return HS_OK;
}

hs_status hs_set_timing_period(hs_sim *s, int period)
{
    if (!s || period < 1) return HS_ERR_ARG;
    s->timing_period = period;
    return HS_OK;
}

hs_status hs_kernel_timing(hs_sim *s, int which, double *avg_ms, int64_t *launches)
{
    if (!s || which < 0 || which >= HS_NUM_KERNELS || !avg_ms) return HS_ERR_ARG;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    double tot = 0.0;
    int64_t n = 0;
    for (const auto &ev : s->events) {
        if (!ev.b[which] || !ev.e[which]) continue;
        float ms = 0.f;
        HIPCHK(s, hipEventElapsedTime(&ms, ev.b[which], ev.e[which]));
        tot += ms;
        ++n;
    }
    *avg_ms = n ? tot / (double)n : 0.0;
    if (launches) *launches = n;
    return HS_OK;
}

static void destroy_events(hs_sim *s)
{
    for (auto &ev : s->events)
        for (int k = 0; k < HS_NUM_KERNELS; ++k) {
            if (ev.b[k]) (void)hipEventDestroy(ev.b[k]);
            if (ev.e[k]) (void)hipEventDestroy(ev.e[k]);
        }
    s->events.clear();
}

hs_status hs_clear_timing(hs_sim *s)
{
    if (!s) return HS_ERR_ARG;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    destroy_events(s);
    s->timed_steps = 0;
    return HS_OK;
}

hs_status hs_autotune(hs_sim *s, int steps_per_trial, hs_tune_report *rep)
{
    if (!s || steps_per_trial < 1) return HS_ERR_ARG;
    if (s->failed) return HS_ERR_STATE;
    hs_status st = check_device(s);
    if (st) return st;
    // candidate blocks per grid of each tunable kernel group
    struct Cand {
        int which;
        std::vector<int> grids;
    };
    const std::vector<Cand> cands = {
        {HS_KERNEL_COLLIDE, {1024, 2048, 3072, 4096, 6144, 8192}},
        {HS_KERNEL_GATHER, {2048, 4096, 8192, 16384}},
        {HS_KERNEL_SCALARS, {2048, 4096, 8192, 16384}},
        // dense cells: a few hundred on the cylinder, tens of thousands on the O-grids
        {HS_KERNEL_DENSE, {128, 256, 512, 1024, 2048}},
        {HS_KERNEL_MOVE, {4096, 8192, 16384, 32768}},
        {HS_KERNEL_SCATTER, {2048, 4096, 8192, 16384}},
    };
    if (s->graph_ready) {                       // shapes change: capture again later
        (void)hipGraphExecDestroy(s->gexec);
        (void)hipGraphDestroy(s->graph);
        s->gexec = nullptr;
        s->graph = nullptr;
        s->graph_ready = false;
    }
    const uint32_t saved = s->timing;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    destroy_events(s);
    hs_tune_report r;
    std::memset(&r, 0, sizeof(r));
    for (const Cand &c : cands) {
        if (!s->plan.any_spatial && (c.which == HS_KERNEL_MOVE || c.which == HS_KERNEL_SCATTER)) continue;
        int best = 0;
        double best_ms = 0.0;
        for (int g : c.grids) {
            s->ctx.grid[c.which] = g;
            s->timing = 1u << c.which;
            for (int k = 0; k < steps_per_trial; ++k) enqueue_step(s, 1);
            r.steps += steps_per_trial;
            HIPCHK(s, hipStreamSynchronize(s->stream));
            st = check_device(s);
            if (st) {
                s->timing = saved;
                destroy_events(s);
                return st;
            }
            double tot = 0.0;
            int n = 0;
            for (const auto &ev : s->events) {
                float ms = 0.f;
                if (ev.b[c.which] && ev.e[c.which] && hipEventElapsedTime(&ms, ev.b[c.which], ev.e[c.which]) == hipSuccess) {
                    tot += ms;
                    ++n;
                }
            }
            destroy_events(s);
            const double avg = n ? tot / n : 0.0;
            if (best == 0 || avg < best_ms) {
                best = g;
                best_ms = avg;
            }
        }
        s->ctx.grid[c.which] = best;
        r.grid[c.which] = best;
        r.ms[c.which] = best_ms;
    }
    s->timing = saved;
    s->timed_steps = 0;
    if (rep) *rep = r;
    return HS_OK;
}

hs_status hs_set_grid(hs_sim *s, int which, int32_t blocks)
{
    if (!s || which < 0 || which >= HS_NUM_KERNELS || blocks < 0) return HS_ERR_ARG;
    if (s->graph_ready) {
        (void)hipGraphExecDestroy(s->gexec);
        (void)hipGraphDestroy(s->graph);
        s->gexec = nullptr;
        s->graph = nullptr;
        s->graph_ready = false;
    }
    s->ctx.grid[which] = blocks;
    return HS_OK;
}


const char *hs_error_string(const hs_sim *s)
{
    if (!s) return "no sim";
    return s->err.empty() ? "ok" : s->err.c_str();
}

void hs_destroy(hs_sim *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->side) (void)hipStreamSynchronize(s->side);
    destroy_events(s);
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    if (s->side) (void)hipStreamDestroy(s->side);
    delete s;
}

hs_status hs_debug_philox(uint64_t seed, uint32_t stream, uint64_t first_entity, uint32_t step, uint32_t draw,
                          int64_t n, void *dev_out, void *hip_stream)
{
    if (!dev_out || n < 0 || stream > 15) return HS_ERR_ARG;
    if (n == 0) return HS_OK;
    Launch::philox(seed, stream, first_entity, step, draw, n, (uint32_t *)dev_out, hip_stream);
    if (hipGetLastError() != hipSuccess) return HS_ERR_DEVICE;
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return HS_ERR_DEVICE;
    return HS_OK;
}

}  // extern "C"
