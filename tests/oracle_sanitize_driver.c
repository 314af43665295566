/*
 * oracle_sanitize_driver.c -- runs the CPU oracle through every public entry point on small
 * cases of each workload shape, for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_oracle_sanitize.py compiles and runs it; any report aborts it).
 *
 * Cases: the 1-D Sod tube (two regions, specular ends), a 0-D batch with per-cell steps, a
 * 2-D cylinder (inflow, outflow, diffuse body, wall sampling, adaptive global step), a jet
 * slot, a 3-D sphere, a quadrilateral box mesh and a hexahedral box mesh with wall, inflow,
 * outflow and specular boundaries.  Sampling starts at step 0 so Step (5)-(6) run too.
 * Exit status 0 when every call succeeds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hs_oracle.h"

#define CHECK(x)                                                                  \
    do {                                                                          \
        int rc_ = (x);                                                            \
        if (rc_ != HSO_OK) {                                                      \
            fprintf(stderr, "%s:%d: %s -> %d\n", __FILE__, __LINE__, #x, rc_);    \
            exit(1);                                                              \
        }                                                                         \
    } while (0)

static const double KB = 1.380649e-23;

static hso_gas argon(void)
{
    hso_gas g = {6.63e-26, 4.17e-10, 273.0, 0.81, 2.117e-5, 2.0 / 3.0, 5.0 / 3.0};
    return g;
}

static hso_case base_case(int dim, int nx, int ny, int nz, double h)
{
    hso_case c;
    memset(&c, 0, sizeof c);
    c.dim = dim;
    c.nx = nx;
    c.ny = ny;
    c.nz = nz;
    for (int a = 0; a < 3; ++a) c.h[a] = (a < dim) ? h : 1.0;
    c.F_N = 1.0;
    c.T_sigma = 1000.0;
    c.seed = 1;
    c.n_steady = 0;
    return c;
}

/* Everything a caller can ask of a case after stepping it. */
static void exercise(hso_sim *s, int c, int n_surf)
{
    const int64_t nc = hso_num_cells(s, c), np = hso_num_particles(s, c);
    double *n = calloc((size_t)nc, sizeof(double)), *u = calloc(3 * (size_t)nc, sizeof(double));
    double *T = calloc((size_t)nc, sizeof(double)), *q = calloc(3 * (size_t)nc, sizeof(double));
    int64_t ns = 0;
    CHECK(hso_sample_moments(s, c, 0, n, u, T, q, &ns));
    CHECK(hso_sample_moments(s, c, 1, n, u, T, q, &ns));
    CHECK(hso_dsmc_ratio(s, c, n));
    hso_trace *tr = calloc((size_t)nc, sizeof(hso_trace));
    CHECK(hso_get_trace(s, c, tr));
    double *vol = calloc((size_t)nc, sizeof(double)), *sig = calloc((size_t)nc, sizeof(double));
    double *acc = calloc(13 * (size_t)nc, sizeof(double));
    CHECK(hso_get_cells(s, c, vol, sig, acc, &ns));
    CHECK(hso_set_cells(s, c, sig, acc, ns));
    double *x = calloc(3 * (size_t)np + 3, sizeof(double)), *v = calloc(3 * (size_t)np + 3, sizeof(double));
    int32_t *cell = calloc((size_t)np + 1, sizeof(int32_t));
    int64_t *id = calloc((size_t)np + 1, sizeof(int64_t));
    int64_t next_id = 0, step = 0;
    CHECK(hso_get_state(s, c, x, v, cell, id, &next_id, &step));
    CHECK(hso_set_state(s, c, np, x, v, cell, id, next_id, step));
    double dt = 0.0, ts = 0.0;
    CHECK(hso_step_dt(s, c, &dt, &ts));
    if (dt > 0.0) CHECK(hso_set_step_dt(s, c, dt, ts));   /* 0-D cases have no global step */
    hso_counters cn;
    CHECK(hso_get_counters(s, c, &cn));
    const int64_t nf = hso_num_faces(s, c);
    if (nf > 0) {
        int32_t *fc = calloc((size_t)nf, sizeof(int32_t)), *fs = calloc((size_t)nf, sizeof(int32_t));
        double *fl = calloc((size_t)nf, sizeof(double));
        CHECK(hso_face_info(s, c, fc, fs, fl));
        free(fc);
        free(fs);
        free(fl);
    }
    if (n_surf > 0) {
        double *sums = calloc(7 * (size_t)n_surf, sizeof(double));
        double *el = calloc(8 * (size_t)n_surf, sizeof(double)), body[5];
        CHECK(hso_get_surface(s, c, sums));
        CHECK(hso_set_surface(s, c, sums));
        CHECK(hso_surface_sample(s, c, el, body, &ns));
        free(sums);
        free(el);
    }
    free(n); free(u); free(T); free(q); free(tr); free(vol); free(sig); free(acc);
    free(x); free(v); free(cell); free(id);
}

static void run(const hso_gas *g, const hso_case *cases, int n_cases, int steps)
{
    hso_sim *s = NULL;
    CHECK(hso_create(g, cases, n_cases, 1, &s));
    CHECK(hso_init_particles(s));
    CHECK(hso_step(s, steps));
    for (int c = 0; c < n_cases; ++c) exercise(s, c, cases[c].n_surf);
    CHECK(hso_step(s, 1));
    for (int c = 0; c < n_cases; ++c) {
        hso_counters cn;
        CHECK(hso_get_counters(s, c, &cn));
        printf("dim %d: %lld particles, %lld injected, %lld accepted, %lld relaxed, %lld wall hits\n",
               cases[c].dim, (long long)hso_num_particles(s, c), (long long)cn.injected, (long long)cn.accepted,
               (long long)cn.relaxed, (long long)cn.wall_hits);
    }
    hso_destroy(s);
}

/* A quadrilateral box mesh of nx x ny cells of size h; edge codes on the four sides. */
static void quad_box(int nx, int ny, double h, const int side[4], hso_mesh *m, double **xy, int32_t **quad,
                     int32_t **nbr)
{
    const int nn = (nx + 1) * (ny + 1), ncl = nx * ny;
    *xy = malloc(2 * (size_t)nn * sizeof(double));
    *quad = malloc(4 * (size_t)ncl * sizeof(int32_t));
    *nbr = malloc(4 * (size_t)ncl * sizeof(int32_t));
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            (*xy)[2 * (j * (nx + 1) + i)] = i * h;
            (*xy)[2 * (j * (nx + 1) + i) + 1] = j * h;
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const int k = j * nx + i, n0 = j * (nx + 1) + i;
            int32_t *q = *quad + 4 * k, *b = *nbr + 4 * k;
            q[0] = n0;
            q[1] = n0 + 1;
            q[2] = n0 + nx + 2;
            q[3] = n0 + nx + 1;
            b[0] = j > 0 ? k - nx : side[2];          /* bottom edge */
            b[1] = i < nx - 1 ? k + 1 : side[1];      /* right edge  */
            b[2] = j < ny - 1 ? k + nx : side[3];     /* top edge    */
            b[3] = i > 0 ? k - 1 : side[0];           /* left edge   */
        }
    m->n_nodes = nn;
    m->n_cells = ncl;
    m->xy = *xy;
    m->quad = *quad;
    m->nbr = *nbr;
}

/* A hexahedral box mesh of n^3 cells of size h; face codes: -x inflow, +x outflow, the rest
 * given by `other`. */
static void hex_box(int n, double h, int other, hso_mesh *m, double **xyz, int32_t **hex, int32_t **nbr)
{
    const int np1 = n + 1, nn = np1 * np1 * np1, ncl = n * n * n;
    *xyz = malloc(3 * (size_t)nn * sizeof(double));
    *hex = malloc(8 * (size_t)ncl * sizeof(int32_t));
    *nbr = malloc(6 * (size_t)ncl * sizeof(int32_t));
    for (int k = 0; k <= n; ++k)
        for (int j = 0; j <= n; ++j)
            for (int i = 0; i <= n; ++i) {
                double *p = *xyz + 3 * ((k * np1 + j) * np1 + i);
                p[0] = i * h;
                p[1] = j * h;
                p[2] = k * h;
            }
#define NODE(i, j, k) (((k) * np1 + (j)) * np1 + (i))
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const int c = (k * n + j) * n + i;
                int32_t *q = *hex + 8 * c, *b = *nbr + 6 * c;
                q[0] = NODE(i, j, k);
                q[1] = NODE(i + 1, j, k);
                q[2] = NODE(i + 1, j + 1, k);
                q[3] = NODE(i, j + 1, k);
                q[4] = NODE(i, j, k + 1);
                q[5] = NODE(i + 1, j, k + 1);
                q[6] = NODE(i + 1, j + 1, k + 1);
                q[7] = NODE(i, j + 1, k + 1);
                /* faces (0,3,2,1) -z, (4,5,6,7) +z, (0,1,5,4) -y, (1,2,6,5) +x, (2,3,7,6) +y,
                 * (3,0,4,7) -x */
                b[0] = k > 0 ? c - n * n : other;
                b[1] = k < n - 1 ? c + n * n : other;
                b[2] = j > 0 ? c - n : other;
                b[3] = i < n - 1 ? c + 1 : HSO_EDGE_OUTFLOW;
                b[4] = j < n - 1 ? c + n : other;
                b[5] = i > 0 ? c - 1 : HSO_EDGE_INFLOW;
            }
#undef NODE
    m->n_nodes = nn;
    m->n_cells = ncl;
    m->xy = *xyz;
    m->quad = *hex;
    m->nbr = *nbr;
}

int main(void)
{
    const hso_gas g = argon();
    const double R = KB / g.m;

    /* building blocks */
    {
        uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
        hso_philox4x32_10(ctr, key, out);
        hso_draw(7, 1, 9, 3, 2, out);
        (void)hso_uniform(out[0]);
        (void)hso_index(out[1], 17);
        (void)hso_sigma_c(&g, 500.0);
        (void)hso_viscosity(&g, 300.0);
        (void)hso_mean_free_path(&g, 1e20, 300.0);
        hso_state st = {1e20, {300.0, 10.0, 0.0}, 250.0};
        const double nrm[3] = {1.0, 0.0, 0.0};
        (void)hso_inflow_number_flux(&g, &st, nrm);
        uint32_t w[4 * 64];
        for (int i = 0; i < 64; ++i) hso_draw(3, 2, (uint64_t)i, 0, 0, w + 4 * i);
        int used = 0;
        (void)hso_sample_normal_speed(0.7, w, 64, &used);
        (void)hso_sample_normal_speed(-0.4, w, 64, &used);
        (void)hso_sample_normal_speed(-1.5, w, 64, &used);
        double v3[3 * 7], U[3], T, Q[3];
        for (int i = 0; i < 21; ++i) v3[i] = 100.0 * sin(1.0 + i) + 37.0 * i;
        CHECK(hso_cell_moments(&g, 7, v3, 1e15, 1e-6, U, &T, Q));
        uint32_t w5[5 * 64];
        for (int i = 0; i < 64; ++i) {
            uint32_t t4[4];
            hso_draw(4, 0, (uint64_t)i, 0, 1, t4);
            memcpy(w5 + 5 * i, t4, sizeof t4);
            w5[5 * i + 4] = t4[0] ^ 0x9E3779B9u;
        }
        double C[3];
        const double p = 1e20 * KB * T;
        (void)hso_shakhov_sample(&g, T, p, Q, 3.0, w5, 64, C);
        double dd, ds;
        hso_split(1e-6, 3e-7, 1e-6, &dd, &ds);
        hso_split(1e-7, 3e-7, 1e-6, &dd, &ds);
    }

    /* 1-D Sod tube: two regions, specular ends */
    {
        hso_case c = base_case(1, 40, 1, 1, 1.0 / 40);
        c.bc[0] = c.bc[1] = HSO_BC_SPECULAR;
        const double boxes[12] = {0, 0, 0, 0.5, 1, 1, 0.5, 0, 0, 1, 1, 1};
        const hso_state sts[2] = {{1.29438e22, {0, 0, 0}, 273.0}, {1.61798e21, {0, 0, 0}, 218.4}};
        c.n_regions = 2;
        c.region_box = boxes;
        c.region_state = sts;
        c.F_N = 1.29438e22 * (1.0 / 40) / 80.0;
        c.dt_G = 0.5 * (1.0 / 40) / sqrt(5.0 / 3.0 * R * 273.0);
        c.T_sigma = 273.0;
        c.capacity = 6000;
        run(&g, &c, 1, 4);
    }

    /* 0-D batch, per-cell dt / tau from 0.01 to 100 */
    {
        hso_case c = base_case(0, 12, 1, 1, 1.0);
        const double box[6] = {0, 0, 0, 0, 0, 0};
        const hso_state st = {1.29438e20, {0, 0, 0}, 273.0};
        double r[12];
        for (int k = 0; k < 12; ++k) r[k] = pow(10.0, -2.0 + 4.0 * k / 11.0);
        c.n_regions = 1;
        c.region_box = box;
        c.region_state = &st;
        c.F_N = 1.29438e20 / 200.0;
        c.T_sigma = 400.0;
        c.dt_over_tau = r;
        c.capacity = 12 * 260;
        run(&g, &c, 1, 3);
    }

    /* 2-D cylinder (inflow -x, +-y; outflow +x; diffuse body; wall sampling) and a jet slot,
     * batched; the cylinder with the adaptive global step */
    {
        const double Uinf = 2634.658009218744, ninf = 1.1753626818345325e20;
        hso_case cs[2];
        const double h = 8.0 / 40;
        cs[0] = base_case(2, 40, 30, 1, h);
        cs[0].bc[0] = cs[0].bc[2] = cs[0].bc[3] = HSO_BC_INFLOW;
        cs[0].inflow = (hso_state){ninf, {Uinf, 0, 0}, 200.0};
        const double box0[6] = {0, 0, 0, 8, 6, 1};
        cs[0].n_regions = 1;
        cs[0].region_box = box0;
        cs[0].region_state = &cs[0].inflow;
        cs[0].body = HSO_BODY_CYLINDER;
        cs[0].body_c[0] = 2.5;
        cs[0].body_c[1] = 3.0;
        cs[0].body_r = 0.5;
        cs[0].body_T = 500.0;
        cs[0].F_N = ninf * h * h / 6.0;
        cs[0].dt_G = h / 2898.1238101406184;
        cs[0].T_sigma = 6866.67;
        cs[0].capacity = 40 * 30 * 12;
        cs[0].n_surf = 18;
        cs[0].adapt_dt = 1;
        const double hj = 1.0 / 20;
        cs[1] = base_case(2, 40, 20, 1, hj);
        cs[1].bc[0] = HSO_BC_INFLOW;
        const double ne = 3e19;
        cs[1].inflow = (hso_state){ne, {279.45, 0, 0}, 225.0};
        cs[1].slot_lo[1] = 0.4;
        cs[1].slot_hi[1] = 0.6;
        cs[1].F_N = ne * hj * hj / 20.0;
        cs[1].dt_G = hj / (2.0 * 279.45);
        cs[1].T_sigma = 300.0;
        cs[1].capacity = 40 * 20 * 30;
        cs[1].seed = 2;
        run(&g, cs, 2, 5);
    }

    /* 3-D sphere */
    {
        const double h = 6.0 / 12, ninf = 1.1753626818345325e20;
        hso_case c = base_case(3, 12, 8, 8, h);
        c.bc[0] = c.bc[2] = c.bc[3] = c.bc[4] = c.bc[5] = HSO_BC_INFLOW;
        c.inflow = (hso_state){ninf, {2634.658009218744, 0, 0}, 200.0};
        const double box[6] = {0, 0, 0, 6, 4, 4};
        c.n_regions = 1;
        c.region_box = box;
        c.region_state = &c.inflow;
        c.body = HSO_BODY_SPHERE;
        c.body_c[0] = c.body_c[1] = c.body_c[2] = 2.0;
        c.body_r = 0.5;
        c.body_T = 500.0;
        c.F_N = ninf * h * h * h / 4.0;
        c.dt_G = h / 2898.1238101406184;
        c.T_sigma = 6866.67;
        c.capacity = 12 * 8 * 8 * 10;
        c.n_surf = 9;
        run(&g, &c, 1, 3);
    }

    /* quadrilateral box mesh: inflow left, outflow right, wall bottom, specular top */
    {
        hso_mesh m;
        double *xy;
        int32_t *quad, *nbr;
        const int side[4] = {HSO_EDGE_INFLOW, HSO_EDGE_OUTFLOW, HSO_EDGE_WALL, HSO_EDGE_SPECULAR};
        quad_box(8, 6, 0.1, side, &m, &xy, &quad, &nbr);
        hso_case c = base_case(2, 1, 1, 1, 0.1);
        c.h[2] = 1.0;
        c.mesh = &m;
        c.inflow = (hso_state){1e20, {800.0, 0, 0}, 300.0};
        const double box[6] = {-1, -1, -1, 2, 2, 2};
        c.n_regions = 1;
        c.region_box = box;
        c.region_state = &c.inflow;
        c.body = HSO_BODY_CYLINDER;
        c.body_c[0] = 0.4;
        c.body_c[1] = -1.0;
        c.body_r = 1.0;
        c.body_T = 400.0;
        c.n_surf = 6;
        c.F_N = 1e20 * 0.01 / 12.0;
        c.dt_G = 0.1 / (800.0 + 3.0 * sqrt(R * 300.0));
        c.T_sigma = 1000.0;
        c.capacity = 48 * 40;
        run(&g, &c, 1, 4);
        free(xy);
        free(quad);
        free(nbr);
    }

    /* hexahedral box mesh: inflow -x, outflow +x, walls elsewhere */
    {
        hso_mesh m;
        double *xyz;
        int32_t *hex, *nbr;
        hex_box(3, 0.1, HSO_EDGE_WALL, &m, &xyz, &hex, &nbr);
        hso_case c = base_case(3, 1, 1, 1, 0.1);
        c.mesh = &m;
        c.inflow = (hso_state){1e20, {800.0, 0, 0}, 300.0};
        const double box[6] = {-1, -1, -1, 2, 2, 2};
        c.n_regions = 1;
        c.region_box = box;
        c.region_state = &c.inflow;
        c.body = HSO_BODY_SPHERE;
        c.body_c[0] = c.body_c[1] = c.body_c[2] = 0.15;
        c.body_r = 1.0;
        c.body_T = 400.0;
        c.n_surf = 6;
        c.F_N = 1e20 * 1e-3 / 10.0;
        c.dt_G = 0.1 / (800.0 + 3.0 * sqrt(R * 300.0));
        c.T_sigma = 1000.0;
        c.capacity = 27 * 40;
        run(&g, &c, 1, 4);
        free(xyz);
        free(hex);
        free(nbr);
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
