/*
 * dlb3_oracle.c -- CPU FP64 reference ("oracle") for the three-dimensional
 * form of the phase-field, solute and heat lattices of the diffuse-interface
 * lattice Boltzmann method of Zhan et al. (arXiv:2209.01444): D3Q7 lattices,
 * the d-general anisotropy a_s and N of Sec. 2, no melt flow.
 *
 * TEST INFRASTRUCTURE ONLY.  Loaded by the test suite; never by the product
 * path.  Shares no code with the GPU library or with the 2-D oracle.
 *
 * Readings (the paper prints its matrices for 2-D lattices only):
 *   - D3Q7 velocities c0 = 0, c1..c3 = +x, +y, +z, c4..c6 = -x, -y, -z,
 *     with cs^2 = 1/4: w0 = 1/4, w1..6 = 1/8.  The relations of Secs. 3.1-3.3
 *     are written for a general lattice sound speed (s1 = 1/[a^2 W0^2/(tau0
 *     cs^2) + 1/2], grad phi = -(s1/cs^2)(sum c f + W0^2 N/tau0), the 1/cs^2
 *     of the solute and heat rates).  cs^2 = 1/3 would leave the D3Q7 rest
 *     weight at zero, which decouples the two checkerboard sublattices; a
 *     growing seed then diverges within a few tens of steps.
 *   - MRT transform rows 1, cx, cy, cz, |c|^2, cx^2 - cy^2, cy^2 - cz^2 with
 *     S = diag(1, s1, s1, s1, 1, 1, 1), as the 2-D lattices relax only the
 *     first moments; with every other rate 1 the choice of second-order rows
 *     does not change Lambda = M^-1 S M.
 *   - The equilibria, sources and auxiliary terms of Secs. 3.1-3.3 carry over
 *     with these weights; no flow (u = 0), so d_t(Cu) = d_t(Hu) = 0.
 *   - Crystal axes along the lattice axes (no orientation).
 *   - Walls (walls = 1): the outermost layer of nodes, rebuilt as a copy of
 *     the inward neighbour (zero gradient), as in the 2-D channel.
 *   - Melt flow (use_ns = 1): D3Q19 (c0 = 0, the six
 *     faces, the twelve edges; w = 1/3, 1/18, 1/36; cs^2 = 1/3) with the
 *     equilibrium, pressure, diffuse force and forcing of Sec. 3.4 (varphi =
 *     0, no external force); MRT in the raw-moment basis 1, c_a, c_a c_b,
 *     c_a^2 c_b, c_a^2 c_b^2 with s2 on the six second-order moments and 1 on
 *     all others, as the 2-D flow lattice; n_sub sub-steps per main step at
 *     the frozen phi of time t, and u = n_sub u' in the solute and heat
 *     equilibria and in d_t(Cu), d_t(Hu) (two-time-scaling, Sec. 4).
 *     With walls, the channel of the 2-D runs in 3-D: the wall nodes'
 *     flow populations are rebuilt by non-equilibrium extrapolation from the
 *     inward neighbour (Sec. 4 preamble), h_b = h^eq(p_b, u_b) + h_f -
 *     h^eq(p_f, u_f): west face x = 0 inlet u_b = u0/n_sub, p_b = p_f; east
 *     face outflow u_b = u_f (its y, z components zeroed where the node also
 *     lies on a y or z wall), p_b = 0; y and z faces free slip (normal
 *     component zeroed), p_b = p_f.  phi, C and H keep the zero-gradient copy
 *     and take the wall node's velocity.
 *
 * Parity status:
 *   anisotropy a_s, N (d-general)                          pinned (closed forms,
 *                                                           finite differences)
 *   phi lattice: modified streaming, source, local gradient pinned (mode decay)
 *   solute / heat lattices: diffusion, conservation        pinned
 *   cubic symmetry of a growing seed                       pinned
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct o3_params {
    int nx, ny, nz;
    int use_t;         /* heat lattice on (else theta = theta0)             */
    int walls;         /* 0 periodic; 1 zero-gradient walls on all faces    */
    int h_quintic;     /* h(phi) = phi (0) or the 15/8 quintic (1)           */
    int c_init_U;      /* initial C from U0 (1) or uniform C0 (0)            */
    int grad_max_iter;
    double W0, tau0, eps4, lambda, Mcinf, k, D, alpha;
    double theta0, U0, C0;
    double seed_R, seed_x, seed_y, seed_z;
    double grad_tol;
    double fixed_as;   /* test hook: > 0 fixes a_s and sets N = 0            */
    int use_ns, n_sub; /* melt flow (periodic only) and its sub-steps        */
    double nu, rho0;   /* viscosity (main-step units) and density            */
    double u0x, u0y, u0z; /* initial velocity (main-step units)             */
} o3_params;

typedef struct o3_state o3_state;

static const int CX[7] = {0, 1, 0, 0, -1, 0, 0};
static const int CY[7] = {0, 0, 1, 0, 0, -1, 0};
static const int CZ[7] = {0, 0, 0, 1, 0, 0, -1};
static const double W7[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
static const double CS2 = 0.25;

static int C19X[19], C19Y[19], C19Z[19];
static double W19[19];
static void init19(void) {
    static const int e[19][3] = {{0, 0, 0},  {1, 0, 0},   {0, 1, 0},  {0, 0, 1},  {-1, 0, 0}, {0, -1, 0}, {0, 0, -1},
                                 {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1},
                                 {1, 0, -1}, {-1, 0, 1},  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    for (int i = 0; i < 19; ++i) {
        C19X[i] = e[i][0];
        C19Y[i] = e[i][1];
        C19Z[i] = e[i][2];
        int n = abs(e[i][0]) + abs(e[i][1]) + abs(e[i][2]);
        W19[i] = n == 0 ? 1.0 / 3.0 : (n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
}

static char g_err[256];
static void set_err(const char* m) {
    strncpy(g_err, m, sizeof g_err - 1);
    g_err[sizeof g_err - 1] = 0;
}
const char* o3_last_error(void) { return g_err; }

/* ---- D3Q7 transform and Lambda = M^-1 S M ---- */
static void m_d3q7(double* M) {
    for (int i = 0; i < 7; ++i) {
        double cx = CX[i], cy = CY[i], cz = CZ[i];
        M[0 * 7 + i] = 1.0;
        M[1 * 7 + i] = cx;
        M[2 * 7 + i] = cy;
        M[3 * 7 + i] = cz;
        M[4 * 7 + i] = cx * cx + cy * cy + cz * cz;
        M[5 * 7 + i] = cx * cx - cy * cy;
        M[6 * 7 + i] = cy * cy - cz * cz;
    }
}

static int invert(const double* A, double* Ainv, int n) {
    double a[400], b[400];
    memcpy(a, A, sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) b[i] = (i / n == i % n) ? 1.0 : 0.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * n + c]) > fabs(a[piv * n + c])) piv = r;
        if (fabs(a[piv * n + c]) < 1e-14) return -1;
        for (int j = 0; j < n; ++j) {
            double t = a[c * n + j]; a[c * n + j] = a[piv * n + j]; a[piv * n + j] = t;
            t = b[c * n + j]; b[c * n + j] = b[piv * n + j]; b[piv * n + j] = t;
        }
        double d = a[c * n + c];
        for (int j = 0; j < n; ++j) { a[c * n + j] /= d; b[c * n + j] /= d; }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = a[r * n + c];
            for (int j = 0; j < n; ++j) { a[r * n + j] -= f * a[c * n + j]; b[r * n + j] -= f * b[c * n + j]; }
        }
    }
    memcpy(Ainv, b, sizeof(double) * n * n);
    return 0;
}

void o3_lambda(double s1, double* L) {
    double M[49], Mi[49], s[7] = {1.0, s1, s1, s1, 1.0, 1.0, 1.0};
    m_d3q7(M);
    invert(M, Mi, 7);
    for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 7; ++j) {
            double acc = 0.0;
            for (int q = 0; q < 7; ++q) acc += Mi[i * 7 + q] * s[q] * M[q * 7 + j];
            L[i * 7 + j] = acc;
        }
}

/* ---- D3Q19 raw-moment transform and Lambda with s2 on the second moments ---- */
static void m_d3q19(double* M, int* second) {
    /* rows: 1; cx cy cz; cx^2 cy^2 cz^2 cxcy cxcz cycz; cx^2cy cx^2cz cy^2cx
     * cy^2cz cz^2cx cz^2cy; cx^2cy^2 cx^2cz^2 cy^2cz^2 */
    for (int i = 0; i < 19; ++i) {
        double x = C19X[i], y = C19Y[i], z = C19Z[i];
        double r[19] = {1, x, y, z, x * x, y * y, z * z, x * y, x * z, y * z, x * x * y, x * x * z, y * y * x,
                        y * y * z, z * z * x, z * z * y, x * x * y * y, x * x * z * z, y * y * z * z};
        for (int q = 0; q < 19; ++q) M[q * 19 + i] = r[q];
    }
    for (int q = 0; q < 19; ++q) second[q] = (q >= 4 && q <= 9);
}

void o3_lambda19(double s2, double* L) {
    init19();
    double M[361], Mi[361];
    int second[19];
    m_d3q19(M, second);
    invert(M, Mi, 19);
    for (int i = 0; i < 19; ++i)
        for (int j = 0; j < 19; ++j) {
            double acc = 0.0;
            for (int q = 0; q < 19; ++q) acc += Mi[i * 19 + q] * (second[q] ? s2 : 1.0) * M[q * 19 + j];
            L[i * 19 + j] = acc;
        }
}

/* h^eq of Sec. 3.4 on D3Q19: sigma_0 = (w0 - 1) p/cs^2 + rho0, sigma_i = w_i p/cs^2,
 * plus w_i [c.u/cs^2 + (c.u)^2/(2 cs^4) - u.u/(2 cs^2)] */
void o3_eq_flow(double rho0, double p, double ux, double uy, double uz, double* o) {
    init19();
    double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < 19; ++i) {
        double cu = C19X[i] * ux + C19Y[i] * uy + C19Z[i] * uz;
        double sig = i == 0 ? (W19[0] - 1.0) * 3.0 * p + rho0 : W19[i] * 3.0 * p;
        o[i] = sig + W19[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Flow macros (Sec. 3.4, sub-step units): u* = sum c h, f = -u*, F_b =
 * [1 - q(phi)] f, u = u* + F_b/2, p = cs^2/(1 - w0) (sum_{i>0} h - w0 |u|^2/(2 cs^2)). */
static void flow_macros3(const double* h, double phi, double* us, double* Fb, double* u, double* pr) {
    double m[3] = {0.0, 0.0, 0.0}, rest = 0.0;
    for (int i = 0; i < 19; ++i) {
        m[0] += C19X[i] * h[i];
        m[1] += C19Y[i] * h[i];
        m[2] += C19Z[i] * h[i];
        if (i) rest += h[i];
    }
    double solid = 1.0 - 0.5 * (1.0 - phi);
    for (int a = 0; a < 3; ++a) {
        us[a] = m[a];
        Fb[a] = solid * (0.0 - m[a]);
        u[a] = us[a] + 0.5 * Fb[a];
    }
    double cs2 = 1.0 / 3.0;
    *pr = cs2 / (1.0 - W19[0]) * (rest - W19[0] * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / (2.0 * cs2));
}

/* ---- anisotropy (Sec. 2), d = 3:
 *   a_s = (1 - 3e)[1 + 4e/(1 - 3e) sum_a n_a^4],  N_a = |g|^2 a_s d a_s/d g_a
 * out: a_s, Nx, Ny, Nz ---- */
void o3_anisotropy(double eps, double gx, double gy, double gz, double* out) {
    double g[3] = {gx, gy, gz};
    double g2 = gx * gx + gy * gy + gz * gz;
    double P = 0.0;
    for (int a = 0; a < 3; ++a) P += g[a] * g[a] * g[a] * g[a];
    double as = (1.0 - 3.0 * eps) * (1.0 + 4.0 * eps / (1.0 - 3.0 * eps) * P / (g2 * g2));
    out[0] = as;
    for (int a = 0; a < 3; ++a) {
        double dsum = 4.0 * g[a] * g[a] * g[a] / (g2 * g2) - 4.0 * g[a] * P / (g2 * g2 * g2);
        out[1 + a] = g2 * as * (4.0 * eps * dsum);
    }
}

static double s1_phi(const o3_params* p, double as) {
    return 1.0 / (as * as * p->W0 * p->W0 / (p->tau0 * CS2) + 0.5);
}
static double s1_solute(const o3_params* p) { return 1.0 / (p->D * (1.0 - p->k) / CS2 + 0.5); }
static double s1_heat(const o3_params* p) { return 1.0 / (p->alpha / CS2 + 0.5); }

/* Local gradient (Sec. 3.1) solved by fixed-point iteration from the
 * isotropic guess, bulk guard |g|^2 < 1e-12.  out: gx, gy, gz, a_s, Nx, Ny,
 * Nz, iterations. */
void o3_local_gradient(const o3_params* p, double m1x, double m1y, double m1z, double* out) {
    double W2t = p->W0 * p->W0 / p->tau0;
    const double a_iso = p->fixed_as > 0 ? p->fixed_as : 1.0;  /* the test hook fixes a_s everywhere */
    double as = a_iso, N[3] = {0.0, 0.0, 0.0};
    double s1 = s1_phi(p, a_iso);
    double g[3] = {-s1 / CS2 * m1x, -s1 / CS2 * m1y, -s1 / CS2 * m1z};
    int it = 0;
    double tol = p->grad_tol > 0 ? p->grad_tol : 1e-14;
    int cap = p->grad_max_iter > 0 ? p->grad_max_iter : 100;
    for (; it < cap; ++it) {
        double gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        if (gg < 1e-12) break;
        double an[4];
        o3_anisotropy(p->eps4, g[0], g[1], g[2], an);
        if (p->fixed_as > 0) { an[0] = p->fixed_as; an[1] = an[2] = an[3] = 0.0; }
        s1 = s1_phi(p, an[0]);
        double m1[3] = {m1x, m1y, m1z}, ng[3], d2 = 0.0, n2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            ng[a] = -s1 / CS2 * (m1[a] + W2t * an[1 + a]);
            d2 += (ng[a] - g[a]) * (ng[a] - g[a]);
            n2 += ng[a] * ng[a];
            g[a] = ng[a];
        }
        if (sqrt(d2) <= tol * sqrt(n2)) { ++it; break; }
    }
    double gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    if (gg < 1e-12) {
        g[0] = g[1] = g[2] = 0.0;
        as = a_iso;
        N[0] = N[1] = N[2] = 0.0;
    } else {
        double an[4];
        o3_anisotropy(p->eps4, g[0], g[1], g[2], an);
        if (p->fixed_as > 0) { an[0] = p->fixed_as; an[1] = an[2] = an[3] = 0.0; }
        as = an[0];
        N[0] = an[1]; N[1] = an[2]; N[2] = an[3];
    }
    out[0] = g[0]; out[1] = g[1]; out[2] = g[2];
    out[3] = as; out[4] = N[0]; out[5] = N[1]; out[6] = N[2]; out[7] = it;
}

static double h_of(double phi, int quintic) {
    if (!quintic) return phi;
    double p2 = phi * phi;
    return 15.0 / 8.0 * (phi - 2.0 * phi * p2 / 3.0 + phi * p2 * p2 / 5.0);
}

/* ---- state ---- */
struct o3_state {
    o3_params p;
    int nx, ny, nz;
    long N;
    double *f, *n, *g, *fn, *nn, *gn;    /* [7][N] */
    double *pf, *pn, *pg, *a2;           /* post-collision, a_s^2 */
    double *phi, *C, *U, *H, *theta;     /* macros of time t */
    double *phi_prev, *Q_prev;
    double *h, *hn, *ph;                 /* flow [19][N] */
    double *u;                           /* [3][N] velocity of time t, main-step units */
    double *Cu_prev, *Hu_prev, *Cu_t, *Hu_t; /* [3][N] */
    int hist_valid;
    long step;
    double L5c[49], L5t[49], L19[361];
};

static double* alloc0(long n) { return (double*)calloc((size_t)n, sizeof(double)); }

o3_state* o3_create(const o3_params* p) {
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) { set_err("grid smaller than 3x3x3"); return NULL; }
    if (p->walls < 0 || p->walls > 1) { set_err("walls must be 0 or 1"); return NULL; }
    if (p->use_ns && (p->n_sub < 1 || !(p->nu > 0))) {
        set_err("melt flow needs n_sub >= 1 and nu > 0");
        return NULL;
    }
    init19();
    double s2 = p->use_ns ? 1.0 / (3.0 * p->nu / p->n_sub + 0.5) : 1.0;
    double rates[4] = {s1_phi(p, 1.0 + p->eps4), s1_solute(p), s1_heat(p), s2};
    for (int i = 0; i < 4; ++i)
        if (!(rates[i] > 0.0 && rates[i] < 2.0)) { set_err("relaxation rate outside (0,2)"); return NULL; }
    o3_state* s = (o3_state*)calloc(1, sizeof(o3_state));
    s->p = *p;
    s->nx = p->nx; s->ny = p->ny; s->nz = p->nz;
    s->N = (long)p->nx * p->ny * p->nz;
    long N = s->N;
    s->f = alloc0(7 * N); s->n = alloc0(7 * N); s->g = alloc0(7 * N);
    s->fn = alloc0(7 * N); s->nn = alloc0(7 * N); s->gn = alloc0(7 * N);
    s->pf = alloc0(7 * N); s->pn = alloc0(7 * N); s->pg = alloc0(7 * N); s->a2 = alloc0(N);
    s->phi = alloc0(N); s->C = alloc0(N); s->U = alloc0(N); s->H = alloc0(N); s->theta = alloc0(N);
    s->phi_prev = alloc0(N); s->Q_prev = alloc0(N);
    s->h = alloc0(19 * N); s->hn = alloc0(19 * N); s->ph = alloc0(19 * N); s->u = alloc0(3 * N);
    s->Cu_prev = alloc0(3 * N); s->Hu_prev = alloc0(3 * N); s->Cu_t = alloc0(3 * N); s->Hu_t = alloc0(3 * N);
    o3_lambda19(s2, s->L19);
    o3_lambda(s1_solute(p), s->L5c);
    o3_lambda(s1_heat(p), s->L5t);
    return s;
}

void o3_destroy(o3_state* s) {
    if (!s) return;
    double* ptrs[] = {s->f, s->n, s->g, s->fn, s->nn, s->gn, s->pf, s->pn, s->pg, s->a2,
                      s->phi, s->C, s->U, s->H, s->theta, s->phi_prev, s->Q_prev, s->h, s->hn, s->ph,
                      s->u, s->Cu_prev, s->Hu_prev, s->Cu_t, s->Hu_t};
    for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) free(ptrs[i]);
    free(s);
}

static inline long id3(const o3_state* s, int x, int y, int z) {
    return ((long)z * s->ny + y) * s->nx + x;
}
static inline int wrap(int a, int n) { return ((a % n) + n) % n; }
static inline int is_wall(const o3_state* s, int x, int y, int z) {
    return s->p.walls && (x == 0 || y == 0 || z == 0 || x == s->nx - 1 || y == s->ny - 1 || z == s->nz - 1);
}
static inline int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }
static long inward(const o3_state* s, int x, int y, int z) {
    return id3(s, clampi(x, 1, s->nx - 2), clampi(y, 1, s->ny - 2), clampi(z, 1, s->nz - 2));
}

static void fill_walls(o3_state* s, double* pop) {
    if (!s->p.walls) return;
    long N = s->N;
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                if (!is_wall(s, x, y, z)) continue;
                long b = id3(s, x, y, z), f = inward(s, x, y, z);
                for (int i = 0; i < 7; ++i) pop[i * N + b] = pop[i * N + f];
            }
}

/* Flow walls by non-equilibrium extrapolation (see the header comment);
 * phi is the frozen phi of the sub-step. */
static void fill_flow_walls3(o3_state* s, double* h, const double* phi) {
    if (!s->p.walls) return;
    const o3_params* p = &s->p;
    long N = s->N;
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                if (!is_wall(s, x, y, z)) continue;
                long b = id3(s, x, y, z), f = inward(s, x, y, z);
                double hf[19], us[3], Fb[3], uf[3], pf;
                for (int i = 0; i < 19; ++i) hf[i] = h[i * N + f];
                flow_macros3(hf, phi[f], us, Fb, uf, &pf);
                double ub[3], pb;
                const int ywall = (y == 0 || y == s->ny - 1), zwall = (z == 0 || z == s->nz - 1);
                if (x == 0) {
                    ub[0] = p->u0x / p->n_sub;
                    ub[1] = p->u0y / p->n_sub;
                    ub[2] = p->u0z / p->n_sub;
                    pb = pf;
                } else if (x == s->nx - 1) {
                    ub[0] = uf[0];
                    ub[1] = ywall ? 0.0 : uf[1];
                    ub[2] = zwall ? 0.0 : uf[2];
                    pb = 0.0;
                } else {
                    ub[0] = uf[0];
                    ub[1] = ywall ? 0.0 : uf[1];
                    ub[2] = zwall ? 0.0 : uf[2];
                    pb = pf;
                }
                double eb[19], ef[19];
                o3_eq_flow(p->rho0, pb, ub[0], ub[1], ub[2], eb);
                o3_eq_flow(p->rho0, pf, uf[0], uf[1], uf[2], ef);
                for (int i = 0; i < 19; ++i) h[i * N + b] = eb[i] + (hf[i] - ef[i]);
            }
}

static void eq_phi(double phi, double* o) { for (int i = 0; i < 7; ++i) o[i] = W7[i] * phi; }
/* n^eq and g^eq of Secs. 3.2, 3.3 with the velocity u (main-step units) */
static void eq_solute(double C, double phi, double U, const double* u, double* o) {
    double qU = 0.5 * (1.0 - phi) * U;
    o[0] = C + (W7[0] - 1.0) * qU;
    for (int i = 1; i < 7; ++i) o[i] = W7[i] * qU + W7[i] * (CX[i] * C * u[0] + CY[i] * C * u[1] + CZ[i] * C * u[2]) / CS2;
}
static void eq_heat(double theta, double phi, int quintic, const double* u, double* o) {
    double H = theta - 0.5 * h_of(phi, quintic);
    o[0] = W7[0] * theta - 0.5 * h_of(phi, quintic);
    for (int i = 1; i < 7; ++i) o[i] = W7[i] * theta + W7[i] * (CX[i] * H * u[0] + CY[i] * H * u[1] + CZ[i] * H * u[2]) / CS2;
}

static void compute_macros(o3_state* s) {
    const o3_params* p = &s->p;
    long N = s->N;
    fill_walls(s, s->f);
    fill_walls(s, s->n);
    if (p->use_t) fill_walls(s, s->g);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; ++x) {
        double ph = 0.0, C = 0.0, H = 0.0;
        for (int i = 0; i < 7; ++i) {
            ph += s->f[i * N + x];
            C += s->n[i * N + x];
            H += s->g[i * N + x];
        }
        s->phi[x] = ph;
        s->C[x] = C;
        s->U[x] = (2.0 * C / (1.0 + p->k - (1.0 - p->k) * ph) - 1.0) / (1.0 - p->k);
        if (p->use_t) {
            s->H[x] = H;
            s->theta[x] = H + 0.5 * h_of(ph, p->h_quintic);
        } else {
            s->theta[x] = p->theta0;
            s->H[x] = p->theta0 - 0.5 * h_of(ph, p->h_quintic);
        }
    }
    /* melt velocity of time t in main-step units: n_sub u' (wall nodes of the
     * flow lattice rebuilt first, with phi of time t) */
    if (p->use_ns) fill_flow_walls3(s, s->h, s->phi);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; ++x) {
        double u[3] = {0.0, 0.0, 0.0};
        if (p->use_ns) {
            double h[19], us[3], Fb[3], pr;
            for (int i = 0; i < 19; ++i) h[i] = s->h[i * N + x];
            flow_macros3(h, s->phi[x], us, Fb, u, &pr);
            for (int a = 0; a < 3; ++a) u[a] *= p->n_sub;
        }
        for (int a = 0; a < 3; ++a) s->u[a * N + x] = u[a];
    }
}

/* Collision at node x (Secs. 3.1-3.3 with the D3Q7 lattice). */
static void collide_node(o3_state* s, long x) {
    const o3_params* p = &s->p;
    long N = s->N;
    double f[7], m1[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 7; ++i) {
        f[i] = s->f[i * N + x];
        m1[0] += CX[i] * f[i];
        m1[1] += CY[i] * f[i];
        m1[2] += CZ[i] * f[i];
    }
    double lg[8];
    o3_local_gradient(p, m1[0], m1[1], m1[2], lg);
    double gx = lg[0], gy = lg[1], gz = lg[2], as = lg[3];
    double a2 = as * as;
    double s1 = s1_phi(p, as);
    double ph = s->phi[x], U = s->U[x], th = s->theta[x];
    double om = 1.0 - ph * ph;
    double Q = ph * om - p->lambda * (th + p->Mcinf * U) * om * om;
    double dQ = 0.0, dphi = 0.0;
    if (s->hist_valid) {
        dQ = Q - s->Q_prev[x];
        dphi = ph - s->phi_prev[x];
    }
    /* phi lattice: S = diag(1, s1, s1, s1, 1, 1, 1) */
    double L[49], feq[7], F[7], dF[7], G[7];
    o3_lambda(s1, L);
    eq_phi(ph, feq);
    for (int i = 0; i < 7; ++i) {
        F[i] = W7[i] * Q / p->tau0;
        dF[i] = W7[i] * dQ / p->tau0;
        G[i] = -W7[i] * (CX[i] * lg[4] + CY[i] * lg[5] + CZ[i] * lg[6]) / a2;
    }
    for (int i = 0; i < 7; ++i) {
        double acc = f[i];
        for (int j = 0; j < 7; ++j) {
            acc -= L[i * 7 + j] * (f[j] - feq[j]);
            acc += ((i == j ? 1.0 : 0.0) - 0.5 * L[i * 7 + j]) * G[j];
        }
        acc += F[i] + 0.5 * a2 * dF[i];
        s->pf[i * N + x] = acc;
    }
    s->a2[x] = a2;
    /* anti-trapping current (Sec. 2) */
    double gn = sqrt(gx * gx + gy * gy + gz * gz), J[3] = {0.0, 0.0, 0.0};
    if (gn > 0.0) {
        double c = -1.0 / (2.0 * sqrt(2.0)) * p->W0 * (1.0 + (1.0 - p->k) * U) * dphi / gn;
        J[0] = c * gx; J[1] = c * gy; J[2] = c * gz;
    }
    /* velocity of time t and the backward differences of C u and H u */
    double u[3] = {s->u[x], s->u[N + x], s->u[2 * N + x]}, dCu[3] = {0.0, 0.0, 0.0}, dHu[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) {
        s->Cu_t[a * N + x] = s->C[x] * u[a];
        s->Hu_t[a * N + x] = s->H[x] * u[a];
        if (s->hist_valid) {
            dCu[a] = s->Cu_t[a * N + x] - s->Cu_prev[a * N + x];
            dHu[a] = s->Hu_t[a * N + x] - s->Hu_prev[a * N + x];
        }
    }
    /* solute lattice (Sec. 3.2): G = w c.[d_t(Cu)/cs^2 + U grad q + J/D] */
    double nv[7], neq[7], GC[7];
    for (int i = 0; i < 7; ++i) nv[i] = s->n[i * N + x];
    eq_solute(s->C[x], ph, U, u, neq);
    double V[3] = {dCu[0] / CS2 + U * (-0.5 * gx) + J[0] / p->D, dCu[1] / CS2 + U * (-0.5 * gy) + J[1] / p->D,
                   dCu[2] / CS2 + U * (-0.5 * gz) + J[2] / p->D};
    for (int i = 0; i < 7; ++i) GC[i] = W7[i] * (CX[i] * V[0] + CY[i] * V[1] + CZ[i] * V[2]);
    for (int i = 0; i < 7; ++i) {
        double acc = nv[i];
        for (int j = 0; j < 7; ++j) {
            acc -= s->L5c[i * 7 + j] * (nv[j] - neq[j]);
            acc += ((i == j ? 1.0 : 0.0) - 0.5 * s->L5c[i * 7 + j]) * GC[j];
        }
        s->pn[i * N + x] = acc;
    }
    /* heat lattice (Sec. 3.3): G = w c.d_t(Hu)/cs^2 */
    if (p->use_t) {
        double gv[7], geq[7], GT[7];
        for (int i = 0; i < 7; ++i) gv[i] = s->g[i * N + x];
        eq_heat(th, ph, p->h_quintic, u, geq);
        for (int i = 0; i < 7; ++i) GT[i] = W7[i] * (CX[i] * dHu[0] + CY[i] * dHu[1] + CZ[i] * dHu[2]) / CS2;
        for (int i = 0; i < 7; ++i) {
            double acc = gv[i];
            for (int j = 0; j < 7; ++j) {
                acc -= s->L5t[i * 7 + j] * (gv[j] - geq[j]);
                acc += ((i == j ? 1.0 : 0.0) - 0.5 * s->L5t[i * 7 + j]) * GT[j];
            }
            s->pg[i * N + x] = acc;
        }
    }
    /* history of time t for the next step */
    s->Q_prev[x] = Q;
}

/* n_sub flow sub-steps (Sec. 3.4) at the frozen phi of time t (s->phi):
 * post = h - Lambda (h - h^eq) + (I - Lambda/2) F, F_i = w_i c_i.F_b/cs^2,
 * then periodic streaming. */
static void flow_substeps(o3_state* s) {
    const o3_params* p = &s->p;
    long N = s->N;
    int nx = s->nx, ny = s->ny, nz = s->nz;
    for (int sub = 0; sub < p->n_sub; ++sub) {
        fill_flow_walls3(s, s->h, s->phi);
#pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) {
            double h[19], us[3], Fb[3], u[3], pr, heq[19], F[19];
            for (int i = 0; i < 19; ++i) h[i] = s->h[i * N + x];
            flow_macros3(h, s->phi[x], us, Fb, u, &pr);
            o3_eq_flow(p->rho0, pr, u[0], u[1], u[2], heq);
            for (int i = 0; i < 19; ++i) F[i] = W19[i] * 3.0 * (C19X[i] * Fb[0] + C19Y[i] * Fb[1] + C19Z[i] * Fb[2]);
            for (int i = 0; i < 19; ++i) {
                double acc = h[i];
                for (int j = 0; j < 19; ++j) {
                    acc -= s->L19[i * 19 + j] * (h[j] - heq[j]);
                    acc += ((i == j ? 1.0 : 0.0) - 0.5 * s->L19[i * 19 + j]) * F[j];
                }
                s->ph[i * N + x] = acc;
            }
        }
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    if (is_wall(s, x, y, z)) continue; /* rebuilt before use */
                    long d = id3(s, x, y, z);
                    for (int i = 0; i < 19; ++i)
                        s->hn[(long)i * N + d] =
                            s->ph[(long)i * N + id3(s, wrap(x - C19X[i], nx), wrap(y - C19Y[i], ny), wrap(z - C19Z[i], nz))];
                }
        double* t = s->h; s->h = s->hn; s->hn = t;
    }
}

int o3_step(o3_state* s, long nsteps) {
    long N = s->N;
    int nx = s->nx, ny = s->ny, nz = s->nz;
    for (long t = 0; t < nsteps; ++t) {
        compute_macros(s);
#pragma omp parallel for schedule(static)
        for (long x = 0; x < N; ++x) collide_node(s, x);
        /* streaming: phi modified (a_s^2 of the collision site), C and H
         * standard; wall nodes are rebuilt before use */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    if (is_wall(s, x, y, z)) continue;
                    long d = id3(s, x, y, z);
                    for (int i = 0; i < 7; ++i) {
                        long src = id3(s, wrap(x - CX[i], nx), wrap(y - CY[i], ny), wrap(z - CZ[i], nz));
                        long o = (long)i * N;
                        s->fn[o + d] = s->f[o + d] + (s->pf[o + src] - s->f[o + d]) / s->a2[src];
                        s->nn[o + d] = s->pn[o + src];
                        if (s->p.use_t) s->gn[o + d] = s->pg[o + src];
                    }
                }
        memcpy(s->phi_prev, s->phi, sizeof(double) * N);
        memcpy(s->Cu_prev, s->Cu_t, sizeof(double) * 3 * N);
        memcpy(s->Hu_prev, s->Hu_t, sizeof(double) * 3 * N);
        double* tmp;
        tmp = s->f; s->f = s->fn; s->fn = tmp;
        tmp = s->n; s->n = s->nn; s->nn = tmp;
        tmp = s->g; s->g = s->gn; s->gn = tmp;
        if (s->p.use_ns) flow_substeps(s);
        s->hist_valid = 1;
        s->step += 1;
    }
    return 0;
}

/* Re-initialise at the given fields (nullable: C from C0/U0, theta0): every
 * lattice at equilibrium, the phi populations with the first moment that
 * makes the local scheme return the isotropic D3Q19 central difference of
 * phi, 3 sum_i w_i c_i phi(x + c_i) (weights 1/18 faces, 1/36 edges;
 * periodic wrap or clamped at the walls): f_i = w_i phi + w_i c_i.m1/cs^2
 * with m1 = -(cs^2/s1) grad phi - W0^2 N/tau0.  History reset. */
int o3_set_fields(o3_state* s, const double* phi, const double* Cin, const double* thin, const double* uxin,
                  const double* uyin, const double* uzin) {
    const o3_params* p = &s->p;
    long N = s->N;
    int nx = s->nx, ny = s->ny, nz = s->nz;
    double W2t = p->W0 * p->W0 / p->tau0;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long id = id3(s, x, y, z);
                double g[3] = {0.0, 0.0, 0.0};
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int nnz = (dx != 0) + (dy != 0) + (dz != 0);
                            if (nnz == 0 || nnz == 3) continue;
                            double w = nnz == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
                            int xx, yy, zz;
                            if (p->walls) {
                                xx = clampi(x + dx, 0, nx - 1); yy = clampi(y + dy, 0, ny - 1); zz = clampi(z + dz, 0, nz - 1);
                            } else {
                                xx = wrap(x + dx, nx); yy = wrap(y + dy, ny); zz = wrap(z + dz, nz);
                            }
                            double v = phi[id3(s, xx, yy, zz)];
                            g[0] += 3.0 * w * dx * v;
                            g[1] += 3.0 * w * dy * v;
                            g[2] += 3.0 * w * dz * v;
                        }
                double V[3] = {0.0, 0.0, 0.0};
                double gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
                if (gg >= 1e-12) {
                    double an[4];
                    o3_anisotropy(p->eps4, g[0], g[1], g[2], an);
                    if (p->fixed_as > 0) { an[0] = p->fixed_as; an[1] = an[2] = an[3] = 0.0; }
                    double s1 = s1_phi(p, an[0]);
                    for (int a = 0; a < 3; ++a) V[a] = -CS2 * g[a] / s1 - W2t * an[1 + a];
                }
                double ph = phi[id];
                double C = Cin ? Cin[id]
                               : (p->c_init_U ? 0.5 * (1.0 + p->k - (1.0 - p->k) * ph) * (1.0 + (1.0 - p->k) * p->U0)
                                              : p->C0);
                double th = thin ? thin[id] : p->theta0;
                double U = (2.0 * C / (1.0 + p->k - (1.0 - p->k) * ph) - 1.0) / (1.0 - p->k);
                double e[7];
                eq_phi(ph, e);
                for (int i = 0; i < 7; ++i)
                    s->f[i * N + id] = e[i] + W7[i] * (CX[i] * V[0] + CY[i] * V[1] + CZ[i] * V[2]) / CS2;
                double u[3] = {uxin ? uxin[id] : p->u0x, uyin ? uyin[id] : p->u0y, uzin ? uzin[id] : p->u0z};
                if (!p->use_ns) u[0] = u[1] = u[2] = 0.0;
                eq_solute(C, ph, U, u, e);
                for (int i = 0; i < 7; ++i) s->n[i * N + id] = e[i];
                eq_heat(th, ph, p->h_quintic, u, e);
                for (int i = 0; i < 7; ++i) s->g[i * N + id] = p->use_t ? e[i] : 0.0;
                if (p->use_ns) {  /* flow at equilibrium with p = 0 and u' = u/n_sub */
                    double hq[19];
                    o3_eq_flow(p->rho0, 0.0, u[0] / p->n_sub, u[1] / p->n_sub, u[2] / p->n_sub, hq);
                    for (int i = 0; i < 19; ++i) s->h[(long)i * N + id] = hq[i];
                }
            }
    s->hist_valid = 0;
    return 0;
}

/* Spherical seed phi = tanh[(R - d)/(sqrt(2) W0)] (Sec. 4), then
 * o3_set_fields with the default C and theta. */
int o3_init_seed(o3_state* s) {
    const o3_params* p = &s->p;
    long N = s->N;
    double* phi = alloc0(N);
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                double dx = x - p->seed_x, dy = y - p->seed_y, dz = z - p->seed_z;
                double d = sqrt(dx * dx + dy * dy + dz * dz);
                phi[id3(s, x, y, z)] = tanh((p->seed_R - d) / (sqrt(2.0) * p->W0));
            }
    int rc = o3_set_fields(s, phi, NULL, NULL, NULL, NULL, NULL);
    free(phi);
    return rc;
}

long o3_step_count(const o3_state* s) { return s->step; }

/* Eight planes of N: phi, C, U, theta, ux, uy, uz (main-step units), p
 * (main-step units, n_sub^2 p'); x fastest, then y, then z. */
int o3_get_fields(o3_state* s, double* out) {
    compute_macros(s);
    long N = s->N;
    memcpy(out, s->phi, sizeof(double) * N);
    memcpy(out + N, s->C, sizeof(double) * N);
    memcpy(out + 2 * N, s->U, sizeof(double) * N);
    memcpy(out + 3 * N, s->theta, sizeof(double) * N);
    memcpy(out + 4 * N, s->u, sizeof(double) * 3 * N);
    for (long x = 0; x < N; ++x) {
        double pr = 0.0;
        if (s->p.use_ns) {
            double h[19], us[3], Fb[3], u[3];
            for (int i = 0; i < 19; ++i) h[i] = s->h[i * N + x];
            flow_macros3(h, s->phi[x], us, Fb, u, &pr);
            pr *= (double)s->p.n_sub * s->p.n_sub;
        }
        out[7 * N + x] = pr;
    }
    return 0;
}

/* out[0..9]: sum C, sum H, solid fraction sum((1 + phi)/2)/N, non-finite
 * count, tip positions along +x, +y, +z, -x, -y, -z from the seed node
 * (rounded centre): the last + to - crossing of phi on the axis, refined
 * linearly in atanh(phi). */
int o3_reduce(o3_state* s, double* out) {
    compute_macros(s);
    long N = s->N;
    double sc = 0.0, sh = 0.0, fs = 0.0, bad = 0.0;
    for (long x = 0; x < N; ++x) {
        sc += s->C[x];
        sh += s->H[x];
        fs += 0.5 * (1.0 + s->phi[x]);
        if (!isfinite(s->phi[x]) || !isfinite(s->C[x]) || !isfinite(s->theta[x])) bad += 1.0;
    }
    out[0] = sc; out[1] = sh; out[2] = fs / (double)N; out[3] = bad;
    int cx = (int)lround(s->p.seed_x), cy = (int)lround(s->p.seed_y), cz = (int)lround(s->p.seed_z);
    const double lim = 1.0 - 1.0 / 1073741824.0;
    for (int arm = 0; arm < 6; ++arm) {
        int i = 1 + arm;
        double best = -1.0, prev = 0.0;
        for (int j = 0;; ++j) {
            int x = cx + j * CX[i], y = cy + j * CY[i], z = cz + j * CZ[i];
            if (x < 0 || y < 0 || z < 0 || x >= s->nx || y >= s->ny || z >= s->nz) break;
            double v = s->phi[id3(s, x, y, z)];
            v = v > lim ? lim : (v < -lim ? -lim : v);
            double ps = atanh(v);
            if (j > 0 && prev > 0.0 && ps <= 0.0) best = (j - 1) + prev / (prev - ps);
            prev = ps;
        }
        out[4 + arm] = best;
    }
    return 0;
}
