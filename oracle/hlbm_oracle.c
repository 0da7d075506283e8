/*
 * hlbm_oracle.c -- plain, slow, FP64 CPU oracle of the homogenized lattice BGK
 * (HLBM) sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: only tests/, the smoke check and the CPU-baseline leg of bench.py
 * use it.  It shares no code, header, table or constant generator with the HIP
 * library; the two agree only through the paper and the written readings of it.
 *
 * What it computes (Simonis et al., "Homogenized lattice Boltzmann methods for
 * fluid flow through porous media -- part I"):
 *   * Kinetic model: the BGK Boltzmann equation (Sec. 3.1, eq:BGKBE) whose
 *     Maxwellian is replaced by the homogenized Maxwellian
 *     M^eq = f^eq(n, varpi*u, T) with porosity control varpi = 1 - nu*tau/K
 *     (Sec. 3.2, eq:porousVeloMaxwellian and eq:d-definition).  Here the caller
 *     gives d = 1 - varpi in [0,1] per cell.
 *   * Moments: density and velocity as zeroth and first velocity moments
 *     (Sec. 3.1, Definition of moments).
 *   * Lattice: the paper's Maxwellian has covariance (1/(3 eps^2)) I
 *     (Sec. 3.3, Step 2, eq:homMaxwellianParametrized), i.e. c_s^2 = 1/3 in
 *     lattice units (eps = 1).  The discrete velocity sets (D2Q9, D3Q19), the
 *     second-order Hermite truncation of the Maxwellian, the Guo forcing term
 *     and halfway bounce-back are textbook lattice Boltzmann pieces; part I of
 *     the paper defers the lattice discretization to its sequel.
 *
 * State convention: populations are stored shifted, g_i = f_i - w_i*rho0, in
 * structure-of-arrays order g[i*N + cell], cell = x + nx*(y + ny*z).  A state
 * array holds the post-collision populations after a completed step; the
 * initial state "from rest" is g = 0.
 *
 * One time step = pull streaming (oracle_stream) followed by collision of every
 * fluid cell (oracle_collide).  The two are separate full-field passes so that
 * each can be read against its definition on its own.
 *
 * Reported moments after n completed steps are those of the post-streaming,
 * pre-collision populations at time n: rho = rho0 + sum g*, j = sum c g*,
 * u = (j + F/2)/rho (Guo's half-force velocity).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_PERIODIC = 0, OR_WALL = 1, OR_INLET_U = 2, OR_OUTLET_RHO = 3 };

typedef struct {
    int q;             /* 9 (planar D2Q9) or 19 (D3Q19) */
    int nx, ny, nz;    /* nz = 1 for q = 9 */
    double tau;        /* BGK relaxation time, > 1/2 */
    double force[3];   /* body-force density F (lattice units) */
    int bc_lo[3];      /* per axis: OR_PERIODIC, OR_WALL, OR_INLET_U, OR_OUTLET_RHO */
    int bc_hi[3];
    double inlet_u[3]; /* prescribed velocity on an OR_INLET_U face */
    double outlet_rho; /* prescribed density on an OR_OUTLET_RHO face */
    double rho0;       /* reference density of the shifted populations */
} oracle_cfg;

/* ------------------------------------------------------------------------ */
/* Velocity sets.                                                            */
/* The set is built from its definition rather than typed in as a table:     */
/* every integer vector with components in {-1,0,1} (third component 0 for   */
/* the planar set) whose squared length is at most 2.  Weights depend on the */
/* squared length only: D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int q;
    int c[19][3];
    double w[19];
    int opp[19];
} lattice_t;

static int build_lattice(int q, lattice_t *L)
{
    double wlen[3];
    int zmax;
    if (q == 9) {
        wlen[0] = 4.0 / 9.0; wlen[1] = 1.0 / 9.0; wlen[2] = 1.0 / 36.0; zmax = 0;
    } else if (q == 19) {
        wlen[0] = 1.0 / 3.0; wlen[1] = 1.0 / 18.0; wlen[2] = 1.0 / 36.0; zmax = 1;
    } else {
        return -1;
    }
    int n = 0;
    for (int cz = -zmax; cz <= zmax; ++cz)
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) {
                int len2 = cx * cx + cy * cy + cz * cz;
                if (len2 > 2) continue;
                L->c[n][0] = cx; L->c[n][1] = cy; L->c[n][2] = cz;
                L->w[n] = wlen[len2];
                ++n;
            }
    if (n != q) return -1;
    L->q = q;
    for (int i = 0; i < q; ++i) {
        L->opp[i] = -1;
        for (int k = 0; k < q; ++k)
            if (L->c[k][0] == -L->c[i][0] && L->c[k][1] == -L->c[i][1] &&
                L->c[k][2] == -L->c[i][2])
                L->opp[i] = k;
    }
    return 0;
}

/* Exported so tests can map between this ordering and any other. */
int oracle_lattice(int q, int *c, double *w)
{
    lattice_t L;
    if (build_lattice(q, &L)) return -1;
    for (int i = 0; i < q; ++i) {
        c[3 * i + 0] = L.c[i][0]; c[3 * i + 1] = L.c[i][1]; c[3 * i + 2] = L.c[i][2];
        w[i] = L.w[i];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers                                                          */
/* ------------------------------------------------------------------------ */
static long cell_index(const oracle_cfg *cfg, int x, int y, int z)
{
    return (long)x + (long)cfg->nx * ((long)y + (long)cfg->ny * (long)z);
}

static void dims(const oracle_cfg *cfg, int n[3])
{
    n[0] = cfg->nx; n[1] = cfg->ny; n[2] = cfg->nz;
}

/* A wall face makes its first (lo) or last (hi) layer of cells solid. */
static int in_wall_layer(const oracle_cfg *cfg, const int s[3])
{
    int n[3];
    dims(cfg, n);
    for (int a = 0; a < 3; ++a) {
        if (cfg->bc_lo[a] == OR_WALL && s[a] == 0) return 1;
        if (cfg->bc_hi[a] == OR_WALL && s[a] == n[a] - 1) return 1;
    }
    return 0;
}

static int is_solid(const oracle_cfg *cfg, int x, int y, int z)
{
    int s[3] = { x, y, z };
    return in_wall_layer(cfg, s);
}

/* Second-order truncated Maxwellian of density rho and velocity u, c_s^2 = 1/3,
 * returned shifted by w_i*rho0:
 *   g_i^eq = w_i * [ (rho - rho0) + rho*(3 c.u + 9/2 (c.u)^2 - 3/2 u.u) ].    */
static void equilibrium(const lattice_t *L, double rho0, double rho, const double u[3],
                        double *geq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L->q; ++i) {
        double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
        geq[i] = L->w[i] * ((rho - rho0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

void oracle_equilibrium(int q, double rho0, double rho, const double *u, double *geq)
{
    lattice_t L;
    if (build_lattice(q, &L)) return;
    equilibrium(&L, rho0, rho, u, geq);
}

/* ------------------------------------------------------------------------ */
/* Collision of one fluid cell (pre-collision g* in, post-collision out).    */
/*   rho = rho0 + sum g*,  j = sum c g*,  u = (j + F/2)/rho                   */
/*   u_eq = (1 - d) u        -- homogenized Maxwellian, varpi = 1 - d         */
/*   g^post = g* - (g* - g^eq(rho, u_eq))/tau + S                            */
/*   S_i = (1 - 1/(2 tau)) w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)]  (Guo)      */
/* ------------------------------------------------------------------------ */
static void collide_cell(const lattice_t *L, const oracle_cfg *cfg, double d,
                         const double *gpre, double *gpost)
{
    const double *F = cfg->force;
    double drho = 0.0, j[3] = { 0.0, 0.0, 0.0 };
    for (int i = 0; i < L->q; ++i) {
        drho += gpre[i];
        for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * gpre[i];
    }
    double rho = cfg->rho0 + drho;
    double u[3], ueq[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = (j[a] + 0.5 * F[a]) / rho;
        ueq[a] = (1.0 - d) * u[a];
    }
    double geq[19];
    equilibrium(L, cfg->rho0, rho, ueq, geq);
    double pref = 1.0 - 0.5 / cfg->tau;
    for (int i = 0; i < L->q; ++i) {
        double cu = 0.0, cF = 0.0, uF = 0.0;
        for (int a = 0; a < 3; ++a) {
            cu += L->c[i][a] * u[a];
            cF += L->c[i][a] * F[a];
            uF += u[a] * F[a];
        }
        double S = pref * L->w[i] * (3.0 * (cF - uF) + 9.0 * cu * cF);
        gpost[i] = gpre[i] - (gpre[i] - geq[i]) / cfg->tau + S;
    }
}

/* Single-cell collision, exported for the moment-property tests. */
int oracle_collide_cell(const oracle_cfg *cfg, double d, const double *gpre, double *gpost)
{
    lattice_t L;
    if (build_lattice(cfg->q, &L)) return -1;
    collide_cell(&L, cfg, d, gpre, gpost);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pull streaming: g*_i(x) = g^post_i(x - c_i).                              */
/*   * periodic axes wrap;                                                   */
/*   * a source cell inside a wall layer is replaced by halfway bounce-back, */
/*     g*_i(x) = g^post_opp(i)(x); this takes precedence on edges;           */
/*   * a source beyond an open face (lowest such axis first) is replaced by   */
/*     an equilibrium built from the cell's own post-collision state:         */
/*       inlet : f^eq(rho_b, u_in) - w rho0, rho_b = rho0 + sum_j g^post_j(x) */
/*       outlet: f^eq(rho_out, u_b) - w rho0, u_b = (sum_j c_j g^post_j(x))/rho_b */
/* Solid cells get zero populations.                                         */
/* ------------------------------------------------------------------------ */
static void stream_cell(const lattice_t *L, const oracle_cfg *cfg, const double *post,
                        double *pre, int x, int y, int z)
{
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    const long cell = cell_index(cfg, x, y, z);
    int n[3];
    dims(cfg, n);
    if (is_solid(cfg, x, y, z)) {
        for (int i = 0; i < L->q; ++i) pre[i * N + cell] = 0.0;
        return;
    }
    int X[3] = { x, y, z };
    for (int i = 0; i < L->q; ++i) {
        int s[3];
        int open_axis = -1, open_side = 0;
        for (int a = 0; a < 3; ++a) {
            s[a] = X[a] - L->c[i][a];
            if (s[a] < 0) {
                if (cfg->bc_lo[a] == OR_PERIODIC) s[a] += n[a];
                else if (open_axis < 0) { open_axis = a; open_side = -1; }
            } else if (s[a] >= n[a]) {
                if (cfg->bc_hi[a] == OR_PERIODIC) s[a] -= n[a];
                else if (open_axis < 0) { open_axis = a; open_side = +1; }
            }
        }
        if (in_wall_layer(cfg, s)) {
            pre[i * N + cell] = post[(long)L->opp[i] * N + cell];
            continue;
        }
        if (open_axis < 0) {
            pre[i * N + cell] = post[(long)i * N + cell_index(cfg, s[0], s[1], s[2])];
            continue;
        }
        int kind = open_side < 0 ? cfg->bc_lo[open_axis] : cfg->bc_hi[open_axis];
        double rho_b = cfg->rho0, jb[3] = { 0.0, 0.0, 0.0 };
        for (int k = 0; k < L->q; ++k) {
            double gk = post[(long)k * N + cell];
            rho_b += gk;
            for (int a = 0; a < 3; ++a) jb[a] += L->c[k][a] * gk;
        }
        double geq[19];
        if (kind == OR_INLET_U) {
            equilibrium(L, cfg->rho0, rho_b, cfg->inlet_u, geq);
        } else { /* OR_OUTLET_RHO */
            double ub[3] = { jb[0] / rho_b, jb[1] / rho_b, jb[2] / rho_b };
            equilibrium(L, cfg->rho0, cfg->outlet_rho, ub, geq);
        }
        pre[i * N + cell] = geq[i];
    }
}

static int check_cfg(const oracle_cfg *cfg, lattice_t *L)
{
    if (build_lattice(cfg->q, L)) return -1;
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return -1;
    if (cfg->q == 9 && cfg->nz != 1) return -1;
    if (!(cfg->tau > 0.5)) return -1;
    for (int a = 0; a < 3; ++a) {
        int lo = cfg->bc_lo[a], hi = cfg->bc_hi[a];
        if ((lo == OR_PERIODIC) != (hi == OR_PERIODIC)) return -1;
        if (lo < 0 || lo > 3 || hi < 0 || hi > 3) return -1;
    }
    return 0;
}

int oracle_stream(const oracle_cfg *cfg, const double *post, double *pre, int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    if (nthreads < 1) nthreads = 1;
    const int ny = cfg->ny, nz = cfg->nz, nx = cfg->nx;
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) stream_cell(&L, cfg, post, pre, x, y, z);
    return 0;
}

int oracle_collide(const oracle_cfg *cfg, const double *d, const double *pre, double *post,
                   int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    if (nthreads < 1) nthreads = 1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    const int ny = cfg->ny, nz = cfg->nz, nx = cfg->nx, q = cfg->q;
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long cell = cell_index(cfg, x, y, z);
                double gin[19], gout[19];
                if (is_solid(cfg, x, y, z)) {
                    for (int i = 0; i < q; ++i) post[i * N + cell] = 0.0;
                    continue;
                }
                for (int i = 0; i < q; ++i) gin[i] = pre[i * N + cell];
                collide_cell(&L, cfg, d[cell], gin, gout);
                for (int i = 0; i < q; ++i) post[i * N + cell] = gout[i];
            }
    return 0;
}

/* Moments of pre-collision populations: drho = rho - rho0 and u = (j + F/2)/rho,
 * u stored as u[a*N + cell].  Solid cells report drho = 0, u = 0.            */
int oracle_moments(const oracle_cfg *cfg, const double *pre, double *drho, double *u)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    for (int z = 0; z < cfg->nz; ++z)
        for (int y = 0; y < cfg->ny; ++y)
            for (int x = 0; x < cfg->nx; ++x) {
                long cell = cell_index(cfg, x, y, z);
                if (is_solid(cfg, x, y, z)) {
                    drho[cell] = 0.0;
                    for (int a = 0; a < 3; ++a) u[a * N + cell] = 0.0;
                    continue;
                }
                double s = 0.0, j[3] = { 0.0, 0.0, 0.0 };
                for (int i = 0; i < L.q; ++i) {
                    double g = pre[i * N + cell];
                    s += g;
                    for (int a = 0; a < 3; ++a) j[a] += L.c[i][a] * g;
                }
                double rho = cfg->rho0 + s;
                drho[cell] = s;
                for (int a = 0; a < 3; ++a) u[a * N + cell] = (j[a] + 0.5 * cfg->force[a]) / rho;
            }
    return 0;
}

/* Advance the post-collision state g by nsteps (g is overwritten). */
int oracle_run(const oracle_cfg *cfg, const double *d, int nsteps, double *g, int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    double *pre = (double *)malloc(sizeof(double) * (size_t)L.q * (size_t)N);
    if (!pre) return -2;
    for (int t = 0; t < nsteps; ++t) {
        oracle_stream(cfg, g, pre, nthreads);
        oracle_collide(cfg, d, pre, g, nthreads);
    }
    free(pre);
    return 0;
}

/* Moments at the current time level of a post-collision state: stream, then
 * take moments (the state itself is not changed).                           */
int oracle_observe(const oracle_cfg *cfg, const double *g, double *drho, double *u,
                   int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    double *pre = (double *)malloc(sizeof(double) * (size_t)L.q * (size_t)N);
    if (!pre) return -2;
    oracle_stream(cfg, g, pre, nthreads);
    oracle_moments(cfg, pre, drho, u);
    free(pre);
    return 0;
}

/* ======================================================================== */
/* Anisotropic porosity control (the tensor-permeability extension the     */
/* paper names as future work; Sec. 3.2 fixes the scalar case by assuming   */
/* isotropy).  The drag (1/tau)(1 - varpi) rho u becomes (1/tau) rho D u    */
/* with D = nu tau K^{-1} a symmetric 3x3 matrix per cell, i.e. the         */
/* equilibrium velocity is u_eq = (I - D) u.  D is passed as 6 rows         */
/* D6[k*N + cell], k = xx, yy, zz, xy, xz, yz.  Everything else is the     */
/* scalar collision above.                                                 */
/* ======================================================================== */
static void tensor_of(const double *D6, long N, long cell, double Dm[3][3])
{
    Dm[0][0] = D6[0 * N + cell];
    Dm[1][1] = D6[1 * N + cell];
    Dm[2][2] = D6[2 * N + cell];
    Dm[0][1] = Dm[1][0] = D6[3 * N + cell];
    Dm[0][2] = Dm[2][0] = D6[4 * N + cell];
    Dm[1][2] = Dm[2][1] = D6[5 * N + cell];
}

static void collide_cell_tensor(const lattice_t *L, const oracle_cfg *cfg, const double Dm[3][3],
                                const double *gpre, double *gpost)
{
    const double *F = cfg->force;
    double drho = 0.0, j[3] = { 0.0, 0.0, 0.0 };
    for (int i = 0; i < L->q; ++i) {
        drho += gpre[i];
        for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * gpre[i];
    }
    double rho = cfg->rho0 + drho;
    double u[3], ueq[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / rho;
    for (int a = 0; a < 3; ++a) {
        double Du = 0.0;
        for (int b = 0; b < 3; ++b) Du += Dm[a][b] * u[b];
        ueq[a] = u[a] - Du;
    }
    double geq[19];
    equilibrium(L, cfg->rho0, rho, ueq, geq);
    double pref = 1.0 - 0.5 / cfg->tau;
    for (int i = 0; i < L->q; ++i) {
        double cu = 0.0, cF = 0.0, uF = 0.0;
        for (int a = 0; a < 3; ++a) {
            cu += L->c[i][a] * u[a];
            cF += L->c[i][a] * F[a];
            uF += u[a] * F[a];
        }
        double S = pref * L->w[i] * (3.0 * (cF - uF) + 9.0 * cu * cF);
        gpost[i] = gpre[i] - (gpre[i] - geq[i]) / cfg->tau + S;
    }
}

int oracle_collide_cell_tensor(const oracle_cfg *cfg, const double *D6cell, const double *gpre,
                               double *gpost)
{
    lattice_t L;
    if (build_lattice(cfg->q, &L)) return -1;
    double Dm[3][3];
    tensor_of(D6cell, 1, 0, Dm);
    collide_cell_tensor(&L, cfg, Dm, gpre, gpost);
    return 0;
}

int oracle_collide_tensor(const oracle_cfg *cfg, const double *D6, const double *pre, double *post,
                          int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    if (nthreads < 1) nthreads = 1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    const int ny = cfg->ny, nz = cfg->nz, nx = cfg->nx, q = cfg->q;
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long cell = cell_index(cfg, x, y, z);
                double gin[19], gout[19], Dm[3][3];
                if (is_solid(cfg, x, y, z)) {
                    for (int i = 0; i < q; ++i) post[i * N + cell] = 0.0;
                    continue;
                }
                for (int i = 0; i < q; ++i) gin[i] = pre[i * N + cell];
                tensor_of(D6, N, cell, Dm);
                collide_cell_tensor(&L, cfg, Dm, gin, gout);
                for (int i = 0; i < q; ++i) post[i * N + cell] = gout[i];
            }
    return 0;
}

int oracle_run_tensor(const oracle_cfg *cfg, const double *D6, int nsteps, double *g, int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    double *pre = (double *)malloc(sizeof(double) * (size_t)L.q * (size_t)N);
    if (!pre) return -2;
    for (int t = 0; t < nsteps; ++t) {
        oracle_stream(cfg, g, pre, nthreads);
        oracle_collide_tensor(cfg, D6, pre, g, nthreads);
    }
    free(pre);
    return 0;
}

/* ======================================================================== */
/* Resolved obstacles: a per-cell solid mask in a fully periodic box.       */
/* The no-slip condition u = 0 on the obstacle surface (Sec. 2.4,            */
/* eq:targetEBTL) by halfway bounce-back at every fluid-solid link: a       */
/* population whose source cell is solid is the cell's own opposite one.     */
/* Solid cells hold zeros and report zero moments.  This is the resolved    */
/* geometry of the unit-cell Stokes problem, the reference the homogenized  */
/* control stands in for.                                                   */
/* ======================================================================== */
static int masked_cfg_ok(const oracle_cfg *cfg, lattice_t *L)
{
    if (check_cfg(cfg, L)) return 0;
    for (int a = 0; a < 3; ++a)
        if (cfg->bc_lo[a] != OR_PERIODIC || cfg->bc_hi[a] != OR_PERIODIC) return 0;
    return 1;
}

int oracle_stream_masked(const oracle_cfg *cfg, const unsigned char *mask, const double *post,
                         double *pre, int nthreads)
{
    lattice_t L;
    if (!masked_cfg_ok(cfg, &L)) return -1;
    if (nthreads < 1) nthreads = 1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    const int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long cell = cell_index(cfg, x, y, z);
                if (mask[cell]) {
                    for (int i = 0; i < L.q; ++i) pre[i * N + cell] = 0.0;
                    continue;
                }
                for (int i = 0; i < L.q; ++i) {
                    int sx = ((x - L.c[i][0]) % nx + nx) % nx;
                    int sy = ((y - L.c[i][1]) % ny + ny) % ny;
                    int sz = ((z - L.c[i][2]) % nz + nz) % nz;
                    const long src = cell_index(cfg, sx, sy, sz);
                    if (mask[src])
                        pre[i * N + cell] = post[(long)L.opp[i] * N + cell];
                    else
                        pre[i * N + cell] = post[(long)i * N + src];
                }
            }
    return 0;
}

int oracle_collide_masked(const oracle_cfg *cfg, const unsigned char *mask, const double *d,
                          const double *pre, double *post, int nthreads)
{
    lattice_t L;
    if (!masked_cfg_ok(cfg, &L)) return -1;
    if (nthreads < 1) nthreads = 1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    const int q = cfg->q;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long cell = 0; cell < N; ++cell) {
        double gin[19], gout[19];
        if (mask[cell]) {
            for (int i = 0; i < q; ++i) post[i * N + cell] = 0.0;
            continue;
        }
        for (int i = 0; i < q; ++i) gin[i] = pre[i * N + cell];
        collide_cell(&L, cfg, d[cell], gin, gout);
        for (int i = 0; i < q; ++i) post[i * N + cell] = gout[i];
    }
    return 0;
}

int oracle_run_masked(const oracle_cfg *cfg, const unsigned char *mask, const double *d, int nsteps,
                      double *g, int nthreads)
{
    lattice_t L;
    if (!masked_cfg_ok(cfg, &L)) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    double *pre = (double *)malloc(sizeof(double) * (size_t)L.q * (size_t)N);
    if (!pre) return -2;
    for (int t = 0; t < nsteps; ++t) {
        oracle_stream_masked(cfg, mask, g, pre, nthreads);
        oracle_collide_masked(cfg, mask, d, pre, g, nthreads);
    }
    free(pre);
    return 0;
}

/* Moments at the time level of post-collision state g with a solid mask. */
int oracle_observe_masked(const oracle_cfg *cfg, const unsigned char *mask, const double *g,
                          double *drho, double *u, int nthreads)
{
    lattice_t L;
    if (!masked_cfg_ok(cfg, &L)) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    double *pre = (double *)malloc(sizeof(double) * (size_t)L.q * (size_t)N);
    if (!pre) return -2;
    oracle_stream_masked(cfg, mask, g, pre, nthreads);
    oracle_moments(cfg, pre, drho, u);   /* solid cells hold zeros: drho = 0 */
    for (long cell = 0; cell < N; ++cell)
        if (mask[cell])
            for (int a = 0; a < 3; ++a) u[a * N + cell] = 0.0;
    free(pre);
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ======================================================================== */
/* Discrete adjoint (reverse mode) of the sweep, for gradients with respect  */
/* to the porosity control d.  The forward map of one step is               */
/*   y_t = S(x_{t-1})  (pull streaming, linear except at open faces)         */
/*   x_t = C(y_t, d)   (cell-local collision)                                */
/* and an objective J observes the moments M(S(x_T)).  The reverse sweep     */
/* applies the transposed Jacobians in the opposite order.  Everything here  */
/* is written from those definitions: the collision's Jacobian is formed    */
/* explicitly, entry by entry, and streaming is transposed as a scatter.     */
/* ======================================================================== */

/* Shifted equilibrium derivatives at (rho, v): d geq_i / d rho and d geq_i / d v_a. */
static void equilibrium_derivs(const lattice_t *L, double rho, const double v[3], int i,
                               double *d_rho, double d_v[3])
{
    double cv = L->c[i][0] * v[0] + L->c[i][1] * v[1] + L->c[i][2] * v[2];
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    *d_rho = L->w[i] * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
    for (int a = 0; a < 3; ++a)
        d_v[a] = L->w[i] * rho * (3.0 * L->c[i][a] + 9.0 * cv * L->c[i][a] - 3.0 * v[a]);
}

/* Transposed collision Jacobian of one fluid cell.  Given the pre-collision
 * populations and the adjoint of the post-collision ones, returns the adjoint
 * of the pre-collision populations and the derivative of <post_bar, post>
 * with respect to d.                                                         */
static void collide_cell_adjoint(const lattice_t *L, const oracle_cfg *cfg, double d,
                                 const double *pre, const double *post_bar, double *pre_bar,
                                 double *d_bar)
{
    const int q = L->q;
    const double *F = cfg->force;
    const double om = 1.0 / cfg->tau, pref = 1.0 - 0.5 / cfg->tau;
    double s = 0.0, j[3] = { 0.0, 0.0, 0.0 };
    for (int i = 0; i < q; ++i) {
        s += pre[i];
        for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * pre[i];
    }
    double rho = cfg->rho0 + s, u[3], v[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = (j[a] + 0.5 * F[a]) / rho;
        v[a] = (1.0 - d) * u[a];
    }
    /* explicit Jacobian J[i][k] = d post_i / d pre_k and Jd[i] = d post_i / d d */
    double J[19][19], Jd[19];
    for (int i = 0; i < q; ++i) {
        double dg_rho, dg_v[3];
        equilibrium_derivs(L, rho, v, i, &dg_rho, dg_v);
        double cF = L->c[i][0] * F[0] + L->c[i][1] * F[1] + L->c[i][2] * F[2];
        double dS_u[3];
        for (int a = 0; a < 3; ++a) dS_u[a] = pref * L->w[i] * (-3.0 * F[a] + 9.0 * L->c[i][a] * cF);
        for (int k = 0; k < q; ++k) {
            double du[3], dv[3];
            for (int a = 0; a < 3; ++a) {
                du[a] = (L->c[k][a] - u[a]) / rho;
                dv[a] = (1.0 - d) * du[a];
            }
            double dgeq = dg_rho + dg_v[0] * dv[0] + dg_v[1] * dv[1] + dg_v[2] * dv[2];
            double dS = dS_u[0] * du[0] + dS_u[1] * du[1] + dS_u[2] * du[2];
            J[i][k] = (i == k ? 1.0 - om : 0.0) + om * dgeq + dS;
        }
        Jd[i] = om * (dg_v[0] * (-u[0]) + dg_v[1] * (-u[1]) + dg_v[2] * (-u[2]));
    }
    double db = 0.0;
    for (int k = 0; k < q; ++k) {
        double acc = 0.0;
        for (int i = 0; i < q; ++i) acc += J[i][k] * post_bar[i];
        pre_bar[k] = acc;
    }
    for (int i = 0; i < q; ++i) db += Jd[i] * post_bar[i];
    *d_bar += db;
}

int oracle_collide_adjoint(const oracle_cfg *cfg, const double *d, const double *pre,
                           const double *post_bar, double *pre_bar, double *d_bar, int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    if (nthreads < 1) nthreads = 1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    const int ny = cfg->ny, nz = cfg->nz, nx = cfg->nx, q = cfg->q;
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long cell = cell_index(cfg, x, y, z);
                if (is_solid(cfg, x, y, z)) {
                    for (int i = 0; i < q; ++i) pre_bar[i * N + cell] = 0.0;
                    continue;
                }
                double gin[19], pb[19], gb[19];
                for (int i = 0; i < q; ++i) {
                    gin[i] = pre[i * N + cell];
                    pb[i] = post_bar[i * N + cell];
                }
                collide_cell_adjoint(&L, cfg, d[cell], gin, pb, gb, &d_bar[cell]);
                for (int i = 0; i < q; ++i) pre_bar[i * N + cell] = gb[i];
            }
    return 0;
}

/* ======================================================================== */
/* Adjoint with the tensor control: u_eq = (I - D) u, D symmetric, given as */
/* its 6 rows (xx, yy, zz, xy, xz, yz).  The collision's Jacobian in the    */
/* populations is the scalar one with (1 - d) replaced by (I - D); its      */
/* Jacobian in the six components follows from d u_eq / d D_ab = -u_b e_a  */
/* for a diagonal entry and -(u_b e_a + u_a e_b) for an off-diagonal one    */
/* (which stands at (a, b) and (b, a)).                                      */
/* ======================================================================== */
static const int TENSOR_AXES[6][2] = { { 0, 0 }, { 1, 1 }, { 2, 2 }, { 0, 1 }, { 0, 2 }, { 1, 2 } };

static void collide_cell_adjoint_tensor(const lattice_t *L, const oracle_cfg *cfg, const double Dm[3][3],
                                        const double *pre, const double *post_bar, double *pre_bar,
                                        double D_bar[6])
{
    const int q = L->q;
    const double *F = cfg->force;
    const double om = 1.0 / cfg->tau, pref = 1.0 - 0.5 / cfg->tau;
    double s = 0.0, j[3] = { 0.0, 0.0, 0.0 };
    for (int i = 0; i < q; ++i) {
        s += pre[i];
        for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * pre[i];
    }
    double rho = cfg->rho0 + s, u[3], v[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / rho;
    for (int a = 0; a < 3; ++a) {
        v[a] = u[a];
        for (int b = 0; b < 3; ++b) v[a] -= Dm[a][b] * u[b];
    }
    /* J[i][k] = d post_i / d pre_k, JD[i][r] = d post_i / d D_r */
    double J[19][19], JD[19][6];
    for (int i = 0; i < q; ++i) {
        double dg_rho, dg_v[3];
        equilibrium_derivs(L, rho, v, i, &dg_rho, dg_v);
        double cF = L->c[i][0] * F[0] + L->c[i][1] * F[1] + L->c[i][2] * F[2];
        double dS_u[3];
        for (int a = 0; a < 3; ++a) dS_u[a] = pref * L->w[i] * (-3.0 * F[a] + 9.0 * L->c[i][a] * cF);
        for (int k = 0; k < q; ++k) {
            double du[3], dv[3];
            for (int a = 0; a < 3; ++a) du[a] = (L->c[k][a] - u[a]) / rho;
            for (int a = 0; a < 3; ++a) {
                dv[a] = du[a];
                for (int b = 0; b < 3; ++b) dv[a] -= Dm[a][b] * du[b];
            }
            double dgeq = dg_rho + dg_v[0] * dv[0] + dg_v[1] * dv[1] + dg_v[2] * dv[2];
            double dS = dS_u[0] * du[0] + dS_u[1] * du[1] + dS_u[2] * du[2];
            J[i][k] = (i == k ? 1.0 - om : 0.0) + om * dgeq + dS;
        }
        for (int r = 0; r < 6; ++r) {
            const int a = TENSOR_AXES[r][0], b = TENSOR_AXES[r][1];
            double dv[3] = { 0.0, 0.0, 0.0 };
            dv[a] -= u[b];
            if (a != b) dv[b] -= u[a];
            JD[i][r] = om * (dg_v[0] * dv[0] + dg_v[1] * dv[1] + dg_v[2] * dv[2]);
        }
    }
    for (int k = 0; k < q; ++k) {
        double acc = 0.0;
        for (int i = 0; i < q; ++i) acc += J[i][k] * post_bar[i];
        pre_bar[k] = acc;
    }
    for (int r = 0; r < 6; ++r) {
        double acc = 0.0;
        for (int i = 0; i < q; ++i) acc += JD[i][r] * post_bar[i];
        D_bar[r] += acc;
    }
}

int oracle_collide_adjoint_tensor(const oracle_cfg *cfg, const double *D6, const double *pre,
                                  const double *post_bar, double *pre_bar, double *D_bar, int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L) || cfg->q != 19) return -1;
    if (nthreads < 1) nthreads = 1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    const int ny = cfg->ny, nz = cfg->nz, nx = cfg->nx, q = cfg->q;
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long cell = cell_index(cfg, x, y, z);
                if (is_solid(cfg, x, y, z)) {
                    for (int i = 0; i < q; ++i) pre_bar[i * N + cell] = 0.0;
                    continue;
                }
                double gin[19], pb[19], gb[19], Dm[3][3], db[6] = { 0, 0, 0, 0, 0, 0 };
                for (int i = 0; i < q; ++i) {
                    gin[i] = pre[i * N + cell];
                    pb[i] = post_bar[i * N + cell];
                }
                tensor_of(D6, N, cell, Dm);
                collide_cell_adjoint_tensor(&L, cfg, Dm, gin, pb, gb, db);
                for (int i = 0; i < q; ++i) pre_bar[i * N + cell] = gb[i];
                for (int r = 0; r < 6; ++r) D_bar[r * N + cell] += db[r];
            }
    return 0;
}

/* Transpose of pull streaming at post-collision state `post`, written as a
 * scatter: every pre-collision population sends its adjoint to whatever it
 * was read from.  post_bar is overwritten.  Single-threaded (scatter).     */
int oracle_stream_adjoint(const oracle_cfg *cfg, const double *post, const double *pre_bar,
                          double *post_bar)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    int n[3];
    dims(cfg, n);
    memset(post_bar, 0, sizeof(double) * (size_t)L.q * (size_t)N);
    for (int z = 0; z < cfg->nz; ++z)
        for (int y = 0; y < cfg->ny; ++y)
            for (int x = 0; x < cfg->nx; ++x) {
                if (is_solid(cfg, x, y, z)) continue;
                const long cell = cell_index(cfg, x, y, z);
                int X[3] = { x, y, z };
                double rho_b = cfg->rho0, jb[3] = { 0.0, 0.0, 0.0 };
                for (int k = 0; k < L.q; ++k) {
                    double gk = post[(long)k * N + cell];
                    rho_b += gk;
                    for (int a = 0; a < 3; ++a) jb[a] += L.c[k][a] * gk;
                }
                for (int i = 0; i < L.q; ++i) {
                    const double gbar = pre_bar[(long)i * N + cell];
                    int s[3];
                    int open_axis = -1, open_side = 0;
                    for (int a = 0; a < 3; ++a) {
                        s[a] = X[a] - L.c[i][a];
                        if (s[a] < 0) {
                            if (cfg->bc_lo[a] == OR_PERIODIC) s[a] += n[a];
                            else if (open_axis < 0) { open_axis = a; open_side = -1; }
                        } else if (s[a] >= n[a]) {
                            if (cfg->bc_hi[a] == OR_PERIODIC) s[a] -= n[a];
                            else if (open_axis < 0) { open_axis = a; open_side = +1; }
                        }
                    }
                    if (in_wall_layer(cfg, s)) {
                        post_bar[(long)L.opp[i] * N + cell] += gbar;
                    } else if (open_axis < 0) {
                        post_bar[(long)i * N + cell_index(cfg, s[0], s[1], s[2])] += gbar;
                    } else {
                        int kind = open_side < 0 ? cfg->bc_lo[open_axis] : cfg->bc_hi[open_axis];
                        if (kind == OR_INLET_U) {
                            /* pre_i = feq_i(rho_b, u_in): depends on every own population via rho_b */
                            double dr, dv[3];
                            equilibrium_derivs(&L, rho_b, cfg->inlet_u, i, &dr, dv);
                            for (int k = 0; k < L.q; ++k) post_bar[(long)k * N + cell] += gbar * dr;
                        } else {
                            /* pre_i = feq_i(rho_out, j_b/rho_b) */
                            double ub[3] = { jb[0] / rho_b, jb[1] / rho_b, jb[2] / rho_b };
                            double dr, dv[3];
                            equilibrium_derivs(&L, cfg->outlet_rho, ub, i, &dr, dv);
                            for (int k = 0; k < L.q; ++k) {
                                double acc = 0.0;
                                for (int a = 0; a < 3; ++a) acc += dv[a] * (L.c[k][a] - ub[a]) / rho_b;
                                post_bar[(long)k * N + cell] += gbar * acc;
                            }
                        }
                    }
                }
            }
    return 0;
}

/* Transpose of the moments observation at pre-collision populations `pre`:
 * pre_bar = d/dpre of sum_cells (drho_bar*drho + u_bar.u).                   */
int oracle_moments_adjoint(const oracle_cfg *cfg, const double *pre, const double *drho_bar,
                           const double *u_bar, double *pre_bar)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    for (int z = 0; z < cfg->nz; ++z)
        for (int y = 0; y < cfg->ny; ++y)
            for (int x = 0; x < cfg->nx; ++x) {
                const long cell = cell_index(cfg, x, y, z);
                if (is_solid(cfg, x, y, z)) {
                    for (int k = 0; k < L.q; ++k) pre_bar[(long)k * N + cell] = 0.0;
                    continue;
                }
                double s = 0.0, j[3] = { 0.0, 0.0, 0.0 };
                for (int k = 0; k < L.q; ++k) {
                    double g = pre[(long)k * N + cell];
                    s += g;
                    for (int a = 0; a < 3; ++a) j[a] += L.c[k][a] * g;
                }
                double rho = cfg->rho0 + s, u[3];
                for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * cfg->force[a]) / rho;
                for (int k = 0; k < L.q; ++k) {
                    double acc = drho_bar[cell];
                    for (int a = 0; a < 3; ++a) acc += u_bar[a * N + cell] * (L.c[k][a] - u[a]) / rho;
                    pre_bar[(long)k * N + cell] = acc;
                }
            }
    return 0;
}

/* Gradient of J = J(moments after nsteps from rest) with respect to d, given
 * dJ/d(drho) and dJ/du at that time level.  Checkpoints every `every` steps
 * and recomputes each segment on the way back.  d_bar is accumulated (+=).  */
int oracle_gradient(const oracle_cfg *cfg, const double *d, int nsteps, int every,
                    const double *drho_bar, const double *u_bar, double *d_bar, int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    if (nsteps < 0 || every < 1) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    const size_t S = (size_t)L.q * (size_t)N;
    const int ncp = nsteps / every + 1;
    double *cps = (double *)calloc((size_t)ncp * S, sizeof(double));
    double *seg = (double *)malloc((size_t)(every + 1) * S * sizeof(double));
    double *pre = (double *)malloc(S * sizeof(double));
    double *xbar = (double *)malloc(S * sizeof(double));
    double *ybar = (double *)malloc(S * sizeof(double));
    double *x = (double *)calloc(S, sizeof(double));
    if (!cps || !seg || !pre || !xbar || !ybar || !x) {
        free(cps); free(seg); free(pre); free(xbar); free(ybar); free(x);
        return -2;
    }
    /* forward with checkpoints: cps[m] = state after m*every steps */
    for (int t = 0; t < nsteps; ++t) {
        if (t % every == 0) memcpy(cps + (size_t)(t / every) * S, x, S * sizeof(double));
        oracle_stream(cfg, x, pre, nthreads);
        oracle_collide(cfg, d, pre, x, nthreads);
    }
    if (nsteps % every == 0) memcpy(cps + (size_t)(nsteps / every) * S, x, S * sizeof(double));
    /* observation adjoint at the final time level */
    oracle_stream(cfg, x, pre, nthreads);
    oracle_moments_adjoint(cfg, pre, drho_bar, u_bar, ybar);
    oracle_stream_adjoint(cfg, x, ybar, xbar);
    /* reverse over segments */
    for (int m = (nsteps - 1) / every; m >= 0 && nsteps > 0; --m) {
        const int t0 = m * every;
        const int t1 = (t0 + every < nsteps) ? t0 + every : nsteps;
        memcpy(seg, cps + (size_t)m * S, S * sizeof(double));
        for (int t = t0; t < t1; ++t) {
            oracle_stream(cfg, seg + (size_t)(t - t0) * S, pre, nthreads);
            oracle_collide(cfg, d, pre, seg + (size_t)(t - t0 + 1) * S, nthreads);
        }
        for (int t = t1; t > t0; --t) {
            /* step t: y_t = S(x_{t-1}), x_t = C(y_t, d) */
            const double *xprev = seg + (size_t)(t - 1 - t0) * S;
            oracle_stream(cfg, xprev, pre, nthreads);
            oracle_collide_adjoint(cfg, d, pre, xbar, ybar, d_bar, nthreads);
            oracle_stream_adjoint(cfg, xprev, ybar, xbar);
        }
    }
    free(cps); free(seg); free(pre); free(xbar); free(ybar); free(x);
    return 0;
}

/* Gradient with respect to the six rows of the tensor control D (D3Q19);
 * otherwise as oracle_gradient.  D_bar[6N] is accumulated (+=).             */
int oracle_gradient_tensor(const oracle_cfg *cfg, const double *D6, int nsteps, int every,
                           const double *drho_bar, const double *u_bar, double *D_bar, int nthreads)
{
    lattice_t L;
    if (check_cfg(cfg, &L) || cfg->q != 19) return -1;
    if (nsteps < 0 || every < 1) return -1;
    const long N = (long)cfg->nx * cfg->ny * cfg->nz;
    const size_t S = (size_t)L.q * (size_t)N;
    const int ncp = nsteps / every + 1;
    double *cps = (double *)calloc((size_t)ncp * S, sizeof(double));
    double *seg = (double *)malloc((size_t)(every + 1) * S * sizeof(double));
    double *pre = (double *)malloc(S * sizeof(double));
    double *xbar = (double *)malloc(S * sizeof(double));
    double *ybar = (double *)malloc(S * sizeof(double));
    double *x = (double *)calloc(S, sizeof(double));
    if (!cps || !seg || !pre || !xbar || !ybar || !x) {
        free(cps); free(seg); free(pre); free(xbar); free(ybar); free(x);
        return -2;
    }
    for (int t = 0; t < nsteps; ++t) {
        if (t % every == 0) memcpy(cps + (size_t)(t / every) * S, x, S * sizeof(double));
        oracle_stream(cfg, x, pre, nthreads);
        oracle_collide_tensor(cfg, D6, pre, x, nthreads);
    }
    oracle_stream(cfg, x, pre, nthreads);
    oracle_moments_adjoint(cfg, pre, drho_bar, u_bar, ybar);
    oracle_stream_adjoint(cfg, x, ybar, xbar);
    for (int m = (nsteps - 1) / every; m >= 0 && nsteps > 0; --m) {
        const int t0 = m * every;
        const int t1 = (t0 + every < nsteps) ? t0 + every : nsteps;
        memcpy(seg, cps + (size_t)m * S, S * sizeof(double));
        for (int t = t0; t < t1; ++t) {
            oracle_stream(cfg, seg + (size_t)(t - t0) * S, pre, nthreads);
            oracle_collide_tensor(cfg, D6, pre, seg + (size_t)(t - t0 + 1) * S, nthreads);
        }
        for (int t = t1; t > t0; --t) {
            const double *xprev = seg + (size_t)(t - 1 - t0) * S;
            oracle_stream(cfg, xprev, pre, nthreads);
            oracle_collide_adjoint_tensor(cfg, D6, pre, xbar, ybar, D_bar, nthreads);
            oracle_stream_adjoint(cfg, xprev, ybar, xbar);
        }
    }
    free(cps); free(seg); free(pre); free(xbar); free(ybar); free(x);
    return 0;
}
