/*
 * dlb_oracle.c -- plain CPU FP64 reference of the diffuse-interface MRT
 * lattice Boltzmann method (Zhan et al., arXiv:2209.01444).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  Shares no
 * code with the GPU library.
 *
 * Written to be checked by eye against the paper:
 *   - populations, not moments: every collision is  f - Lambda (f - f^eq)
 *     + source terms, with Lambda = M^-1 S M formed from the transform
 *     matrices printed in Appendix B and inverted here by Gauss-Jordan;
 *   - equilibria, sources and auxiliary terms exactly as defined in
 *     Sec. 3.1-3.4, evaluated in the order documented beside each one;
 *   - one main step in Jacobi order: every lattice reads the macroscopic
 *     fields of time t; the flow lattice runs n_sub sub-steps with phi frozen
 *     at phi^t (two-time-scaling, Sec. 4 preamble).
 * Readings of points the paper leaves open are marked "Reading:".
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no FMA
 * contraction, so the documented evaluation order is the rounding order).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "dlb_oracle.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static char g_err[256];
const char* orc_last_error(void) { return g_err; }
static void set_err(const char* m) { snprintf(g_err, sizeof g_err, "%s", m); }

/* ---------------------------------------------------------------------------
 * Lattices (Appendix B).  Velocity order = column order of M.
 * ------------------------------------------------------------------------- */
static const int C5X[5] = {0, 1, 0, -1, 0};
static const int C5Y[5] = {0, 0, 1, 0, -1};
static const int C9X[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int C9Y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* Weights.  Not printed in the paper.  D2Q5: the second-moment condition
 * sum_i c_i c_i f_i^eq = C cs^2 I of Appendix A with f^eq = w_i phi and
 * cs^2 = 1/3 forces 2 w_1 = 1/3.  D2Q9: the set that reproduces the printed
 * equilibrium moment vector m_h^eq of Appendix B. */
static const double W5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
static const double W9[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Transform matrices as printed in Appendix B (row-major). */
static const double M5[25] = {
    1, 1, 1, 1, 1,
    0, 1, 0, -1, 0,
    0, 0, 1, 0, -1,
    0, 1, 0, 1, 0,
    0, 0, 1, 0, 1};
static const double M9[81] = {
    1, 1, 1, 1, 1, 1, 1, 1, 1,
    0, 1, 0, -1, 0, 1, -1, -1, 1,
    0, 0, 1, 0, -1, 1, 1, -1, -1,
    0, 1, 0, 1, 0, 1, 1, 1, 1,
    0, 0, 1, 0, 1, 1, 1, 1, 1,
    0, 0, 0, 0, 0, 1, -1, 1, -1,
    0, 0, 0, 0, 0, 1, 1, -1, -1,
    0, 0, 0, 0, 0, 1, -1, -1, 1,
    0, 0, 0, 0, 0, 1, 1, 1, 1};

void orc_m_d2q5(double* out) { memcpy(out, M5, sizeof M5); }
void orc_m_d2q9(double* out) { memcpy(out, M9, sizeof M9); }

/* Gauss-Jordan inverse with partial pivoting of an n x n matrix. */
static int invert(int n, const double* A, double* Ainv) {
    double a[81 * 2];
    int w = 2 * n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < w; ++j)
            a[i * w + j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * w + c]) > fabs(a[piv * w + c])) piv = r;
        if (a[piv * w + c] == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < w; ++j) {
                double t = a[c * w + j];
                a[c * w + j] = a[piv * w + j];
                a[piv * w + j] = t;
            }
        double d = a[c * w + c];
        for (int j = 0; j < w; ++j) a[c * w + j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = a[r * w + c];
            if (f != 0.0)
                for (int j = 0; j < w; ++j) a[r * w + j] -= f * a[c * w + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = a[i * w + n + j];
    return 0;
}

static double M5inv[25], M9inv[81];
static int g_inv_ready = 0;
static void ensure_inverses(void) {
    if (g_inv_ready) return;
    invert(5, M5, M5inv);
    invert(9, M9, M9inv);
    g_inv_ready = 1;
}

/* Lambda = M^-1 S M (Appendix B). */
static void lambda_of(int n, const double* M, const double* Minv, const double* s, double* L) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += Minv[i * n + k] * s[k] * M[k * n + j];
            L[i * n + j] = acc;
        }
}

void orc_lambda_d2q5(double s0, double s1, double s2, double* L) {
    ensure_inverses();
    double s[5] = {s0, s1, s1, s2, s2};
    lambda_of(5, M5, M5inv, s, L);
}

void orc_lambda_d2q9(const double* s9, double* L) {
    ensure_inverses();
    lambda_of(9, M9, M9inv, s9, L);
}

/* ---------------------------------------------------------------------------
 * Equilibria (Sec. 3.1-3.4).  Evaluation order is part of the contract: the
 * GPU library's equilibrium functions evaluate the same expressions in the
 * same order with contraction disabled, so FP64 results agree bit for bit.
 * ------------------------------------------------------------------------- */

/* Sec. 3.1: f_i^eq = w_i phi. */
void orc_eq_phi(double phi, double* out) {
    for (int i = 0; i < 5; ++i) out[i] = W5[i] * phi;
}

/* h(phi) of Sec. 2: phi, or the quintic 15(phi - 2phi^3/3 + phi^5/5)/8. */
static double h_of(double phi, int quintic) {
    if (!quintic) return phi;
    double p2 = phi * phi;
    return 15.0 * (phi - 2.0 * phi * p2 / 3.0 + phi * p2 * p2 / 5.0) / 8.0;
}

/* Sec. 3.2: n_0^eq = C + (w_0 - 1) q U;  n_i^eq = w_i q U + w_i c_i.(C u)/cs^2,
 * q = (1 - phi)/2.  Order: q = 0.5*(1.0-phi); qU = q*U; Cux = C*ux;
 * Cuy = C*uy; cu = cx*Cux + cy*Cuy; n_i = w_i*qU + w_i*(3.0*cu). */
void orc_eq_solute(double C, double phi, double U, double ux, double uy, double* out) {
    double q = 0.5 * (1.0 - phi);
    double qU = q * U;
    double Cux = C * ux, Cuy = C * uy;
    out[0] = C + (W5[0] - 1.0) * qU;
    for (int i = 1; i < 5; ++i) {
        double cu = C5X[i] * Cux + C5Y[i] * Cuy;
        out[i] = W5[i] * qU + W5[i] * (3.0 * cu);
    }
}

/* Sec. 3.3: g_0^eq = w_0 theta - h/2;  g_i^eq = w_i theta + w_i c_i.(H u)/cs^2,
 * H = theta - h/2.  Order: hp = h(phi); H = theta - 0.5*hp; Hux = H*ux;
 * Huy = H*uy; g_0 = w_0*theta - 0.5*hp; g_i = w_i*theta + w_i*(3.0*cu). */
void orc_eq_heat(double theta, double phi, int quintic, double ux, double uy, double* out) {
    double hp = h_of(phi, quintic);
    double H = theta - 0.5 * hp;
    double Hux = H * ux, Huy = H * uy;
    out[0] = W5[0] * theta - 0.5 * hp;
    for (int i = 1; i < 5; ++i) {
        double cu = C5X[i] * Hux + C5Y[i] * Huy;
        out[i] = W5[i] * theta + W5[i] * (3.0 * cu);
    }
}

/* Sec. 3.4: h_i^eq = sigma_i + w_i [c_i.u/cs^2 + uu:(c_i c_i - cs^2 I)/(2cs^4)],
 * sigma_0 = (w_0 - 1) p/cs^2 + rho0, sigma_i = w_i p/cs^2.  Order:
 * uu = ux*ux + uy*uy; cu = cx*ux + cy*uy; sigma_0 = (w_0-1.0)*(3.0*p) + rho0;
 * sigma_i = w_i*(3.0*p); h_i = sigma_i + w_i*(3.0*cu + 4.5*cu*cu - 1.5*uu). */
void orc_eq_flow(double rho0, double p, double ux, double uy, double* out) {
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double cu = C9X[i] * ux + C9Y[i] * uy;
        double sigma = i == 0 ? (W9[0] - 1.0) * (3.0 * p) + rho0 : W9[i] * (3.0 * p);
        out[i] = sigma + W9[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Sec. 3.4 forcing distribution with the adjustable parameter varphi = 0
 * (Sec. 4 preamble): F_i = w_i c_i.F / cs^2. */
void orc_force_flow(double Fx, double Fy, double* out) {
    for (int i = 0; i < 9; ++i) out[i] = W9[i] * (3.0 * (C9X[i] * Fx + C9Y[i] * Fy));
}

/* Sec. 3.4 forcing distribution in full:
 *   F_i = w_i { c_i.G / cs^2 + varphi (uF + Fu):(c_i c_i - cs^2 I) / (2 cs^4) }
 * with G = F + [1 - q(phi)] f; (uF + Fu):(cc - cs^2 I) = 2 (c.u)(c.F) - 2 cs^2 u.F. */
void orc_force_flow_full(double Gx, double Gy, double Fx, double Fy, double ux, double uy,
                         double varphi, double* out) {
    const double cs2 = 1.0 / 3.0;
    for (int i = 0; i < 9; ++i) {
        double cG = C9X[i] * Gx + C9Y[i] * Gy;
        double cu = C9X[i] * ux + C9Y[i] * uy, cF = C9X[i] * Fx + C9Y[i] * Fy;
        double uF = ux * Fx + uy * Fy;
        out[i] = W9[i] * (cG / cs2 + varphi * (2.0 * cu * cF - 2.0 * cs2 * uF) / (2.0 * cs2 * cs2));
    }
}

/* ---------------------------------------------------------------------------
 * Anisotropy (Sec. 2): a_s(n) = (1-3e)[1 + 4e/(1-3e) sum_a n_a^4],
 * n = -grad(phi)/|grad(phi)|;  N_a = |grad phi|^2 a_s d a_s / d(d_a phi).
 * Written from the d-general definition: the derivative of sum g_a^4/|g|^4 is
 * taken term by term.  Reading: a crystal orientation `orient` rotates the
 * gradient into the crystal frame first, and N back out (the paper's runs
 * use orient = 0, where the rotation is the identity).
 * ------------------------------------------------------------------------- */
void orc_anisotropy(double eps, double orient, double gx, double gy, double* out) {
    double co = cos(orient), so = sin(orient);
    double g[2] = {co * gx + so * gy, -so * gx + co * gy}; /* R(-orient) g */
    double g2 = g[0] * g[0] + g[1] * g[1];
    double P = 0.0;
    for (int a = 0; a < 2; ++a) P += g[a] * g[a] * g[a] * g[a];
    double sum_n4 = P / (g2 * g2);
    double as = (1.0 - 3.0 * eps) * (1.0 + 4.0 * eps / (1.0 - 3.0 * eps) * sum_n4);
    double Nc[2];
    for (int a = 0; a < 2; ++a) {
        /* d(sum_n4)/dg_a = 4 g_a^3/|g|^4 - 4 g_a P/|g|^6 */
        double dsum = 4.0 * g[a] * g[a] * g[a] / (g2 * g2) - 4.0 * g[a] * P / (g2 * g2 * g2);
        double das = (1.0 - 3.0 * eps) * (4.0 * eps / (1.0 - 3.0 * eps)) * dsum;
        Nc[a] = g2 * as * das;
    }
    out[0] = as;
    out[1] = co * Nc[0] - so * Nc[1]; /* R(orient) N' */
    out[2] = so * Nc[0] + co * Nc[1];
}

/* ---------------------------------------------------------------------------
 * Local gradient of Sec. 3.1 (general form: Appendix A, local scheme):
 *   grad phi = -(s1/(cs^2 dt)) (sum_i c_i f_i + W0^2 N / tau0),
 *   s1 = 1/[a_s^2 W0^2/(tau0 cs^2 dt) + 1/2].
 * N and s1 depend on grad phi, so the relation is implicit.
 * Reading: solved by fixed-point iteration from the isotropic guess
 * (a_s = 1, N = 0) until |g_new - g| <= tol |g_new| (cap grad_max_iter).
 * Bulk guard: |g|^2 < 1e-12 gives g = 0, a_s = 1, N = 0 (the normal is
 * undefined there).
 * ------------------------------------------------------------------------- */
#define GRAD_GUARD 1e-12

/* heat sub-steps per main step (multi-time-scaling), at least one */
static int heat_sub(const orc_params* p) { return p->n_sub_t > 1 ? p->n_sub_t : 1; }

static double s1_phi(const orc_params* p, double as) {
    double W2t = p->W0 * p->W0 / p->tau0;
    return 1.0 / (as * as * W2t * 3.0 + 0.5);
}

static void aniso_or_hook(const orc_params* p, double gx, double gy, double* a, double* Nx, double* Ny) {
    if (p->fixed_as > 0.0) {
        *a = p->fixed_as;
        *Nx = 0.0;
        *Ny = 0.0;
        return;
    }
    double o[3];
    orc_anisotropy(p->eps4, p->orient, gx, gy, o);
    *a = o[0];
    *Nx = o[1];
    *Ny = o[2];
}

void orc_local_gradient(const orc_params* p, double m1x, double m1y, double* out) {
    double W2t = p->W0 * p->W0 / p->tau0;
    double s1 = s1_phi(p, p->fixed_as > 0.0 ? p->fixed_as : 1.0);
    double gx = -3.0 * s1 * m1x, gy = -3.0 * s1 * m1y;
    int it = 0;
    double a = 1.0, Nx = 0.0, Ny = 0.0;
    int maxit = p->grad_max_iter > 0 ? p->grad_max_iter : 100;
    double tol = p->grad_tol > 0.0 ? p->grad_tol : 1e-14;
    while (it < maxit) {
        if (gx * gx + gy * gy < GRAD_GUARD) break;
        aniso_or_hook(p, gx, gy, &a, &Nx, &Ny);
        s1 = s1_phi(p, a);
        double nx = -3.0 * s1 * (m1x + W2t * Nx);
        double ny = -3.0 * s1 * (m1y + W2t * Ny);
        double d = sqrt((nx - gx) * (nx - gx) + (ny - gy) * (ny - gy));
        gx = nx;
        gy = ny;
        ++it;
        if (d <= tol * sqrt(gx * gx + gy * gy)) break;
    }
    if (gx * gx + gy * gy < GRAD_GUARD) {
        gx = gy = 0.0;
        a = p->fixed_as > 0.0 ? p->fixed_as : 1.0;
        Nx = Ny = 0.0;
    } else {
        aniso_or_hook(p, gx, gy, &a, &Nx, &Ny);
    }
    out[0] = gx;
    out[1] = gy;
    out[2] = a;
    out[3] = Nx;
    out[4] = Ny;
    out[5] = (double)it;
}

/* Isotropic nine-point gradient of a node field: with the D2Q9 weights w_i
 * and cs^2 = 1/3, grad F = (1/cs^2) sum_i w_i c_i F(x + c_i) + O(dx^2).
 * Neighbours wrap on periodic grids and are clamped on channel grids. */
void orc_stencil_gradient(const orc_params* p, const double* F, int x, int y, double* out) {
    int nx = p->nx, ny = p->ny;
    double gx = 0.0, gy = 0.0;
    for (int i = 1; i < 9; ++i) {
        int xx = x + C9X[i], yy = y + C9Y[i];
        if (p->walls) {
            xx = xx < 0 ? 0 : (xx > nx - 1 ? nx - 1 : xx);
            yy = yy < 0 ? 0 : (yy > ny - 1 ? ny - 1 : yy);
        } else {
            xx = (xx % nx + nx) % nx;
            yy = (yy % ny + ny) % ny;
        }
        gx += 3.0 * W9[i] * C9X[i] * F[yy * nx + xx];
        gy += 3.0 * W9[i] * C9Y[i] * F[yy * nx + xx];
    }
    out[0] = gx;
    out[1] = gy;
}

/* ---------------------------------------------------------------------------
 * Flow lattice macros and collision (Sec. 3.4), in sub-step units dt' = 1.
 *   u* = sum c_i h_i + dt/2 F   (external force F = 0, reading)
 *   f  = (u_s - u*)/dt'         (u_s = 0: the dendrite does not move)
 *   u  = u* + dt/2 [1 - q(phi)] f
 *   p  = cs^2/(1-w0) (sum_{i!=0} h_i - w0 u.u/(2cs^2))   (varphi = 0)
 * ------------------------------------------------------------------------- */
static double s2_flow(const orc_params* p);

/* External force of the flow sub-steps: F / N_sub^2 (an acceleration, from
 * main-step to sub-step units). */
static void sub_force(const orc_params* p, double* F) {
    double n = p->use_ns ? (double)p->n_sub : 1.0;
    F[0] = p->force_x / (n * n);
    F[1] = p->force_y / (n * n);
}

/* Sec. 3.4 macroscopic quantities (sub-step units, dt' = 1):
 *   u* = sum c_i h_i + F/2,  f = (u_s - u*)/dt' with u_s = 0,
 *   u = u* + [1 - q(phi)] f / 2,
 *   p = cs^2/(1 - w0) (sum_{i>0} h_i - w0 |u|^2/(2 cs^2) + varphi K u.F / cs^2),
 *   K = 2 (s2 - 3 s4 + s2 s4) / (9 s2 s4)  (Appendix B), s4 = 1. */
static void flow_macros(const orc_params* p, const double* h, double phi, double* ustar, double* Fb,
                        double* u, double* pr) {
    double mx = 0.0, my = 0.0, rest = 0.0, F[2];
    for (int i = 0; i < 9; ++i) {
        mx += C9X[i] * h[i];
        my += C9Y[i] * h[i];
        if (i) rest += h[i];
    }
    sub_force(p, F);
    ustar[0] = mx + 0.5 * F[0];
    ustar[1] = my + 0.5 * F[1];
    double qt = 0.5 * (1.0 - phi);
    double fx = (0.0 - ustar[0]) / 1.0, fy = (0.0 - ustar[1]) / 1.0;
    Fb[0] = (1.0 - qt) * fx;
    Fb[1] = (1.0 - qt) * fy;
    u[0] = ustar[0] + 0.5 * Fb[0];
    u[1] = ustar[1] + 0.5 * Fb[1];
    double cs2 = 1.0 / 3.0;
    double s2 = s2_flow(p), s4 = 1.0;
    double K = 2.0 * (s2 - 3.0 * s4 + s2 * s4) / (9.0 * s2 * s4);
    *pr = cs2 / (1.0 - W9[0]) *
          (rest - W9[0] * (u[0] * u[0] + u[1] * u[1]) / (2.0 * cs2) +
           p->varphi * K * (u[0] * F[0] + u[1] * F[1]) / cs2);
}

typedef struct {
    double L9[81];
    double L5c[25], L5t[25];
} lambdas;

static void collide_flow_node(const orc_params* p, const double* L9, const double* h, double phi,
                              double* post, double* aux) {
    double us[2], Fb[2], u[2], pr, Fe[2];
    flow_macros(p, h, phi, us, Fb, u, &pr);
    sub_force(p, Fe);
    double heq[9], F[9];
    orc_eq_flow(p->rho0, pr, u[0], u[1], heq);
    orc_force_flow_full(Fe[0] + Fb[0], Fe[1] + Fb[1], Fe[0], Fe[1], u[0], u[1], p->varphi, F);
    for (int i = 0; i < 9; ++i) {
        double acc = h[i];
        for (int j = 0; j < 9; ++j) {
            acc -= L9[i * 9 + j] * (h[j] - heq[j]);
            acc += ((i == j ? 1.0 : 0.0) - 0.5 * L9[i * 9 + j]) * F[j];
        }
        post[i] = acc;
    }
    if (aux) {
        aux[0] = us[0];
        aux[1] = us[1];
        aux[2] = u[0];
        aux[3] = u[1];
    }
}

static double s2_flow(const orc_params* p) {
    /* Sec. 4: s2^u = 1/(nu/(cs^2 dt') + 1/2), nu' = nu/N in sub-step units */
    double nu_sub = p->nu / (double)p->n_sub;
    return 1.0 / (3.0 * nu_sub + 0.5);
}

static void flow_lambda(const orc_params* p, double* L9) {
    double s2 = s2_flow(p);
    /* S^u = diag(s0, s1, s1, s2, s2, s2, s3, s3, s4); the others are 1 (Sec. 4) */
    double s[9] = {1.0, 1.0, 1.0, s2, s2, s2, 1.0, 1.0, 1.0};
    orc_lambda_d2q9(s, L9);
}

void orc_collide_flow(const orc_params* p, const double* h, double phi, double* post, double* aux) {
    double L9[81];
    flow_lambda(p, L9);
    collide_flow_node(p, L9, h, phi, post, aux);
}

/* ---------------------------------------------------------------------------
 * State
 * ------------------------------------------------------------------------- */
struct orc_state {
    orc_params p;
    int nx, ny, N;
    double *f, *n, *g, *fn, *nn, *gn; /* [5][N] */
    double *h, *hn;                    /* [9][N] */
    double *phi_prev, *Q_prev, *Cu_prev, *Hu_prev; /* history at t-1 */
    int hist_valid;
    long step;
    /* work arrays */
    double *phi, *C, *H, *theta, *U, *ux, *uy, *Q, *Cu, *Hu, *a2, *pf, *pn, *pg, *ph;
    lambdas L;
};

static double* alloc0(size_t n) { return (double*)calloc(n, sizeof(double)); }

long orc_step_count(const orc_state* s) { return s->step; }

orc_state* orc_create(const orc_params* p) {
    ensure_inverses();
    if (p->nx < 3 || p->ny < 3) {
        set_err("grid smaller than 3x3");
        return NULL;
    }
    if (p->use_ns && p->n_sub < 1) {
        set_err("n_sub < 1");
        return NULL;
    }
    if (p->walls < 0 || p->walls > 2) {
        set_err("walls must be 0, 1 or 2");
        return NULL;
    }
    if (p->walls == 2 && (p->use_ns || p->grad_stencil || heat_sub(p) > 1 || p->phi_static)) {
        set_err("far-field walls need the flow lattice off, the local gradient, one heat step "
                "and a moving phi");
        return NULL;
    }
    double s1 = s1_phi(p, 1.0);
    double s1c = 1.0 / (3.0 * p->D * (1.0 - p->k) + 0.5);
    /* multi-time-scaling of the heat lattice: n_sub_t sub-steps of dt/n_sub_t,
     * diffusivity alpha/n_sub_t per sub-step (reading) */
    double s1t = 1.0 / (3.0 * p->alpha / heat_sub(p) + 0.5);
    double rates[4] = {s1, p->use_c ? s1c : 1.0, p->use_t ? s1t : 1.0, p->use_ns ? s2_flow(p) : 1.0};
    for (int i = 0; i < 4; ++i)
        if (!(rates[i] > 0.0 && rates[i] < 2.0)) {
            set_err("relaxation rate outside (0,2)");
            return NULL;
        }
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    s->p = *p;
    s->nx = p->nx;
    s->ny = p->ny;
    s->N = p->nx * p->ny;
    size_t N = (size_t)s->N;
    s->f = alloc0(5 * N); s->fn = alloc0(5 * N);
    s->n = alloc0(5 * N); s->nn = alloc0(5 * N);
    s->g = alloc0(5 * N); s->gn = alloc0(5 * N);
    s->h = alloc0(9 * N); s->hn = alloc0(9 * N);
    s->phi_prev = alloc0(N); s->Q_prev = alloc0(N);
    s->Cu_prev = alloc0(2 * N); s->Hu_prev = alloc0(2 * N);
    s->phi = alloc0(N); s->C = alloc0(N); s->H = alloc0(N); s->theta = alloc0(N);
    s->U = alloc0(N); s->ux = alloc0(N); s->uy = alloc0(N); s->Q = alloc0(N);
    s->Cu = alloc0(2 * N); s->Hu = alloc0(2 * N); s->a2 = alloc0(N);
    s->pf = alloc0(5 * N); s->pn = alloc0(5 * N); s->pg = alloc0(5 * N); s->ph = alloc0(9 * N);
    orc_lambda_d2q5(1.0, s1c, 1.0, s->L.L5c);
    orc_lambda_d2q5(1.0, s1t, 1.0, s->L.L5t);
    flow_lambda(p, s->L.L9);
    return s;
}

void orc_destroy(orc_state* s) {
    if (!s) return;
    double* ptrs[] = {s->f, s->fn, s->n, s->nn, s->g, s->gn, s->h, s->hn, s->phi_prev, s->Q_prev,
                      s->Cu_prev, s->Hu_prev, s->phi, s->C, s->H, s->theta, s->U, s->ux, s->uy,
                      s->Q, s->Cu, s->Hu, s->a2, s->pf, s->pn, s->pg, s->ph};
    for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) free(ptrs[i]);
    free(s);
}

static inline int wrap(int a, int n) { return ((a % n) + n) % n; }
static inline int is_wall(const orc_state* s, int x, int y) {
    return s->p.walls && (x == 0 || y == 0 || x == s->nx - 1 || y == s->ny - 1);
}
/* inward neighbour of a wall node (diagonal at corners) */
static inline int inward(const orc_state* s, int x, int y) {
    int xf = x < 1 ? 1 : (x > s->nx - 2 ? s->nx - 2 : x);
    int yf = y < 1 ? 1 : (y > s->ny - 2 ? s->ny - 2 : y);
    return yf * s->nx + xf;
}

/* Reading: the walls of the channel configuration are lattice nodes on the
 * outermost ring.  Their populations are rebuilt from the inward neighbour
 * x_f each time they are needed (before every collision and every macro
 * evaluation) by non-equilibrium extrapolation (Sec. 4 preamble):
 *   f(x_b) = f^eq(Psi_b, u_b) + [f(x_f) - f^eq(Psi_f, u_f)].
 * walls = 1, phi, C, H lattices: zero gradient Psi_b = Psi_f with u_b = u_f,
 * which makes the rebuild a copy of x_f's populations.
 * walls = 2, far field (Sec. 4.4: Dirichlet phi = -1, U = U0, theta = theta0
 * on the outer boundary): Psi_b is the far-field liquid, phi = -1 with the C
 * of the initial far field and theta0, at u = 0 (the flow lattice is off in
 * this configuration).  lattice: 0 phi, 1 C, 2 H. */
static double far_field_C(const orc_params* p) {
    /* the initial C at phi = -1: uniform C0, or the C of U = U0 */
    return p->c_init_U ? 0.5 * (1.0 + p->k + (1.0 - p->k)) * (1.0 + (1.0 - p->k) * p->U0) : p->C0;
}
static void fill_cde_walls(orc_state* s, double* pop, int lattice) {
    if (!s->p.walls) return;
    const orc_params* p = &s->p;
    const size_t N = (size_t)s->N;
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            if (!is_wall(s, x, y)) continue;
            int b = y * s->nx + x, f = inward(s, x, y);
            double d[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (p->walls == 2) {
                double phf = 0.0, Cf = 0.0, Hf = 0.0, eb[5], ef[5];
                for (int i = 0; i < 5; ++i) {
                    phf += s->f[i * N + f];
                    if (p->use_c) Cf += s->n[i * N + f];
                    if (p->use_t) Hf += s->g[i * N + f];
                }
                if (lattice == 0) {
                    orc_eq_phi(-1.0, eb);
                    orc_eq_phi(phf, ef);
                } else if (lattice == 1) {
                    double Cb = far_field_C(p);
                    double Ub = (2.0 * Cb / (1.0 + p->k - (1.0 - p->k) * -1.0) - 1.0) / (1.0 - p->k);
                    double Uf = (2.0 * Cf / (1.0 + p->k - (1.0 - p->k) * phf) - 1.0) / (1.0 - p->k);
                    orc_eq_solute(Cb, -1.0, Ub, 0.0, 0.0, eb);
                    orc_eq_solute(Cf, phf, Uf, 0.0, 0.0, ef);
                } else {
                    double thf = Hf + 0.5 * h_of(phf, p->h_quintic);
                    orc_eq_heat(p->theta0, -1.0, p->h_quintic, 0.0, 0.0, eb);
                    orc_eq_heat(thf, phf, p->h_quintic, 0.0, 0.0, ef);
                }
                for (int i = 0; i < 5; ++i) d[i] = eb[i] - ef[i];
            }
            for (int i = 0; i < 5; ++i) pop[(size_t)i * N + b] = pop[(size_t)i * N + f] + d[i];
        }
}

/* Flow lattice walls.  West x=0 (corners included): velocity inlet
 * u_b = u_in/N_sub, p_b = p_f.  East x=nx-1: outflow du/dx = 0 (u_b = u_f)
 * with p_b = 0; at its corners u_b = (u_f,x, 0).  North/south: free slip
 * u_b = (u_f,x, 0), p_b = p_f.  phi is the frozen phi of this sub-step. */
static void fill_flow_walls(orc_state* s, double* h, const double* phi) {
    if (!s->p.walls) return;
    int N = s->N;
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            if (!is_wall(s, x, y)) continue;
            int b = y * s->nx + x, f = inward(s, x, y);
            double hf[9], us[2], Fb[2], uf[2], pf;
            for (int i = 0; i < 9; ++i) hf[i] = h[(size_t)i * N + f];
            flow_macros(&s->p, hf, phi[f], us, Fb, uf, &pf);
            double ub[2], pb;
            if (x == 0) {
                ub[0] = s->p.u_in_x / s->p.n_sub;
                ub[1] = s->p.u_in_y / s->p.n_sub;
                pb = pf;
            } else if (x == s->nx - 1) {
                ub[0] = uf[0];
                ub[1] = (y == 0 || y == s->ny - 1) ? 0.0 : uf[1];
                pb = 0.0;
            } else {
                ub[0] = uf[0];
                ub[1] = 0.0;
                pb = pf;
            }
            double eb[9], ef[9];
            orc_eq_flow(s->p.rho0, pb, ub[0], ub[1], eb);
            orc_eq_flow(s->p.rho0, pf, uf[0], uf[1], ef);
            for (int i = 0; i < 9; ++i) h[(size_t)i * N + b] = eb[i] + (hf[i] - ef[i]);
        }
}

/* Macroscopic fields of time t at every node (Sec. 3.1-3.4):
 * phi = sum f; C = sum n, U from C and phi; theta = sum g + h(phi)/2;
 * u (main-step units) = N_sub * corrected flow velocity with phi^t. */
static void compute_macros(orc_state* s) {
    const orc_params* p = &s->p;
    int N = s->N;
    fill_cde_walls(s, s->f, 0);
    if (p->use_c) fill_cde_walls(s, s->n, 1);
    if (p->use_t) fill_cde_walls(s, s->g, 2);
#pragma omp parallel for schedule(static)
    for (int x = 0; x < N; ++x) {
        double ph = 0.0, C = 0.0, H = 0.0;
        for (int i = 0; i < 5; ++i) ph += s->f[(size_t)i * N + x];
        s->phi[x] = ph;
        if (p->use_c) {
            for (int i = 0; i < 5; ++i) C += s->n[(size_t)i * N + x];
            /* U = [2C/(1+k-(1-k)phi) - 1]/(1-k)  (Sec. 3.2, macro relation) */
            s->C[x] = C;
            s->U[x] = (2.0 * C / (1.0 + p->k - (1.0 - p->k) * ph) - 1.0) / (1.0 - p->k);
        } else {
            s->U[x] = p->U0;
            s->C[x] = 0.5 * (1.0 + p->k - (1.0 - p->k) * ph) * (1.0 + (1.0 - p->k) * p->U0);
        }
        if (p->use_t) {
            for (int i = 0; i < 5; ++i) H += s->g[(size_t)i * N + x];
            s->H[x] = H;
            s->theta[x] = H + 0.5 * h_of(ph, p->h_quintic);
        } else {
            s->theta[x] = p->theta0;
            s->H[x] = p->theta0 - 0.5 * h_of(ph, p->h_quintic);
        }
    }
    if (p->use_ns) {
        fill_flow_walls(s, s->h, s->phi);
#pragma omp parallel for schedule(static)
        for (int x = 0; x < N; ++x) {
            double hx[9], us[2], Fb[2], u[2], pr;
            for (int i = 0; i < 9; ++i) hx[i] = s->h[(size_t)i * N + x];
            flow_macros(p, hx, s->phi[x], us, Fb, u, &pr);
            s->ux[x] = p->n_sub * u[0];
            s->uy[x] = p->n_sub * u[1];
        }
    } else {
        memset(s->ux, 0, sizeof(double) * N);
        memset(s->uy, 0, sizeof(double) * N);
    }
}

/* One main step of the phi, C and theta lattices (Sec. 3.1-3.3) at node x,
 * writing post-collision populations and a_s^2. */
static void collide_pct_node(orc_state* s, int x) {
    const orc_params* p = &s->p;
    int N = s->N;
    double f[5], ph = s->phi[x];
    for (int i = 0; i < 5; ++i) f[i] = s->f[(size_t)i * N + x];
    double m1x = 0.0, m1y = 0.0;
    for (int i = 0; i < 5; ++i) {
        m1x += C5X[i] * f[i];
        m1y += C5Y[i] * f[i];
    }
    double lg[6];
    if (p->grad_stencil) {
        /* ablation: grad phi from the node values of phi at time t; a wall
         * node, a copy of its inward neighbour, takes that node's gradient */
        int xi = x % s->nx, yi = x / s->nx;
        if (is_wall(s, xi, yi)) {
            int f = inward(s, xi, yi);
            xi = f % s->nx;
            yi = f / s->nx;
        }
        orc_stencil_gradient(p, s->phi, xi, yi, lg);
        if (lg[0] * lg[0] + lg[1] * lg[1] < GRAD_GUARD) {
            lg[0] = lg[1] = 0.0;
            lg[2] = p->fixed_as > 0.0 ? p->fixed_as : 1.0;
            lg[3] = lg[4] = 0.0;
        } else {
            aniso_or_hook(p, lg[0], lg[1], &lg[2], &lg[3], &lg[4]);
        }
    } else {
        orc_local_gradient(p, m1x, m1y, lg);
    }
    double gx = lg[0], gy = lg[1], a = lg[2], Nx = lg[3], Ny = lg[4];
    double a2 = a * a;
    double s1 = s1_phi(p, a);
    double U = s->U[x], theta = s->theta[x], C = s->C[x], H = s->H[x];
    double ux = s->ux[x], uy = s->uy[x];

    /* Sec. 2 coupling source */
    double om = 1.0 - ph * ph;
    double Q = ph * om - p->lambda * (theta + p->Mcinf * U) * om * om;
    /* Reading: time derivatives are first-order backward differences over one
     * main step, zero on the first step after (re-)initialisation. */
    double dQ = s->hist_valid ? Q - s->Q_prev[x] : 0.0;
    double dphi = s->hist_valid ? ph - s->phi_prev[x] : 0.0;
    double Cu[2] = {C * ux, C * uy}, Hu[2] = {H * ux, H * uy};
    double dCu[2] = {0, 0}, dHu[2] = {0, 0};
    if (s->hist_valid) {
        dCu[0] = Cu[0] - s->Cu_prev[x];
        dCu[1] = Cu[1] - s->Cu_prev[N + x];
        dHu[0] = Hu[0] - s->Hu_prev[x];
        dHu[1] = Hu[1] - s->Hu_prev[N + x];
    }
    s->Q[x] = Q;
    s->Cu[x] = Cu[0];
    s->Cu[N + x] = Cu[1];
    s->Hu[x] = Hu[0];
    s->Hu[N + x] = Hu[1];

    /* ---- phi lattice, Sec. 3.1 ---- */
    double L[25];
    orc_lambda_d2q5(1.0, s1, 1.0, L);
    double feq[5], F[5], dF[5], G[5];
    orc_eq_phi(ph, feq);
    for (int i = 0; i < 5; ++i) {
        F[i] = W5[i] * Q / p->tau0;
        dF[i] = W5[i] * dQ / p->tau0;
        G[i] = -W5[i] * (C5X[i] * Nx + C5Y[i] * Ny) / a2;
    }
    for (int i = 0; i < 5; ++i) {
        double acc = f[i];
        for (int j = 0; j < 5; ++j) {
            acc -= L[i * 5 + j] * (f[j] - feq[j]);
            acc += ((i == j ? 1.0 : 0.0) - 0.5 * L[i * 5 + j]) * G[j];
        }
        acc += F[i] + 0.5 * a2 * dF[i];
        s->pf[(size_t)i * N + x] = acc;
    }
    s->a2[x] = a2;

    double gnorm = sqrt(gx * gx + gy * gy);
    /* anti-trapping current, Sec. 2 */
    double Jat[2] = {0.0, 0.0};
    if (gnorm > 0.0) {
        double c = -1.0 / (2.0 * sqrt(2.0)) * p->W0 * (1.0 + (1.0 - p->k) * U) * dphi / gnorm;
        Jat[0] = c * gx;
        Jat[1] = c * gy;
    }

    /* ---- solute lattice, Sec. 3.2 ---- */
    if (p->use_c) {
        double nv[5], neq[5], GC[5];
        for (int i = 0; i < 5; ++i) nv[i] = s->n[(size_t)i * N + x];
        orc_eq_solute(C, ph, U, ux, uy, neq);
        /* grad q(phi) = -grad(phi)/2 */
        double Vx = 3.0 * dCu[0] + U * (-0.5 * gx) + Jat[0] / p->D;
        double Vy = 3.0 * dCu[1] + U * (-0.5 * gy) + Jat[1] / p->D;
        for (int i = 0; i < 5; ++i) GC[i] = W5[i] * (C5X[i] * Vx + C5Y[i] * Vy);
        for (int i = 0; i < 5; ++i) {
            double acc = nv[i];
            for (int j = 0; j < 5; ++j) {
                acc -= s->L.L5c[i * 5 + j] * (nv[j] - neq[j]);
                acc += ((i == j ? 1.0 : 0.0) - 0.5 * s->L.L5c[i * 5 + j]) * GC[j];
            }
            s->pn[(size_t)i * N + x] = acc;
        }
    }
    /* ---- heat lattice, Sec. 3.3 (here unless it takes sub-steps) ---- */
    if (p->use_t && heat_sub(p) == 1) {
        double gv[5], geq[5], GT[5];
        for (int i = 0; i < 5; ++i) gv[i] = s->g[(size_t)i * N + x];
        orc_eq_heat(theta, ph, p->h_quintic, ux, uy, geq);
        for (int i = 0; i < 5; ++i) GT[i] = W5[i] * (3.0 * (C5X[i] * dHu[0] + C5Y[i] * dHu[1]));
        for (int i = 0; i < 5; ++i) {
            double acc = gv[i];
            for (int j = 0; j < 5; ++j) {
                acc -= s->L.L5t[i * 5 + j] * (gv[j] - geq[j]);
                acc += ((i == j ? 1.0 : 0.0) - 0.5 * s->L.L5t[i * 5 + j]) * GT[j];
            }
            s->pg[(size_t)i * N + x] = acc;
        }
    }
}

static void swap_ptr(double** a, double** b) {
    double* t = *a;
    *a = *b;
    *b = t;
}

static void flow_substeps(orc_state* s);

/* Heat lattice in n_sub_t sub-steps of dt' = dt/n_sub_t (multi-time-scaling,
 * reading): phi frozen at phi^t as for the flow sub-steps; per sub-step the
 * diffusivity is alpha/n_sub_t (in the relaxation rate), the advecting
 * velocity u^t/n_sub_t, and the correction G = (1/2) c.d_t'(H u') takes the
 * main step's backward difference of H u in sub-step units,
 * d_t(H u)/n_sub_t^2, in every sub-step.  Walls: zero gradient, as for one
 * step. */
static void heat_substeps(orc_state* s) {
    const orc_params* p = &s->p;
    int N = s->N, nx = s->nx, ny = s->ny;
    const int ns = heat_sub(p);
    for (int sub = 0; sub < ns; ++sub) {
        fill_cde_walls(s, s->g, 2);
#pragma omp parallel for schedule(static)
        for (int x = 0; x < N; ++x) {
            double gv[5], geq[5], GT[5], H = 0.0;
            for (int i = 0; i < 5; ++i) {
                gv[i] = s->g[(size_t)i * N + x];
                H += gv[i];
            }
            double ph = s->phi[x];
            double theta = H + 0.5 * h_of(ph, p->h_quintic);
            double dHu[2] = {0.0, 0.0};
            if (s->hist_valid) {
                dHu[0] = (s->Hu[x] - s->Hu_prev[x]) / ((double)ns * ns);
                dHu[1] = (s->Hu[N + x] - s->Hu_prev[N + x]) / ((double)ns * ns);
            }
            orc_eq_heat(theta, ph, p->h_quintic, s->ux[x] / ns, s->uy[x] / ns, geq);
            for (int i = 0; i < 5; ++i) GT[i] = W5[i] * (3.0 * (C5X[i] * dHu[0] + C5Y[i] * dHu[1]));
            for (int i = 0; i < 5; ++i) {
                double acc = gv[i];
                for (int j = 0; j < 5; ++j) {
                    acc -= s->L.L5t[i * 5 + j] * (gv[j] - geq[j]);
                    acc += ((i == j ? 1.0 : 0.0) - 0.5 * s->L.L5t[i * 5 + j]) * GT[j];
                }
                s->pg[(size_t)i * N + x] = acc;
            }
        }
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (is_wall(s, x, y)) continue;
                int d = y * nx + x;
                for (int i = 0; i < 5; ++i) {
                    int src = wrap(y - C5Y[i], ny) * nx + wrap(x - C5X[i], nx);
                    s->gn[(size_t)i * N + d] = s->pg[(size_t)i * N + src];
                }
            }
        swap_ptr(&s->g, &s->gn);
    }
}

static void main_step(orc_state* s) {
    const orc_params* p = &s->p;
    int N = s->N, nx = s->nx, ny = s->ny;
    compute_macros(s);
    if (p->phi_static) {
        /* frozen diffuse solid (Sec. 4.1): only the flow lattice steps */
        if (p->use_ns) flow_substeps(s);
        s->step += 1;
        return;
    }

#pragma omp parallel for schedule(static)
    for (int x = 0; x < N; ++x) collide_pct_node(s, x);

    /* Streaming.  phi lattice: modified streaming of Remark 2 / Sec. 3.1,
     *   f_i(x+c_i,t+1) = f_i(x+c_i,t) + [post_i(x) - f_i(x+c_i,t)] / a_s^2(x)
     * (Reading: a_s^2 is the collision site's).  C and H: standard. */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int d = y * nx + x;
            if (is_wall(s, x, y)) continue; /* rebuilt before use */
            for (int i = 0; i < 5; ++i) {
                int sx = wrap(x - C5X[i], nx), sy = wrap(y - C5Y[i], ny);
                int src = sy * nx + sx;
                size_t o = (size_t)i * N;
                s->fn[o + d] = s->f[o + d] + (s->pf[o + src] - s->f[o + d]) / s->a2[src];
                if (p->use_c) s->nn[o + d] = s->pn[o + src];
                if (p->use_t && heat_sub(p) == 1) s->gn[o + d] = s->pg[o + src];
            }
        }
    swap_ptr(&s->f, &s->fn);
    swap_ptr(&s->n, &s->nn);
    if (heat_sub(p) == 1)
        swap_ptr(&s->g, &s->gn);
    else if (p->use_t)
        heat_substeps(s);

    /* history <- time-t values */
    memcpy(s->phi_prev, s->phi, sizeof(double) * N);
    memcpy(s->Q_prev, s->Q, sizeof(double) * N);
    memcpy(s->Cu_prev, s->Cu, sizeof(double) * 2 * N);
    memcpy(s->Hu_prev, s->Hu, sizeof(double) * 2 * N);

    /* Flow lattice: n_sub sub-steps with phi frozen at phi^t (Sec. 3.4,
     * two-time-scaling of Sec. 4). */
    if (p->use_ns) flow_substeps(s);
    s->hist_valid = 1;
    s->step += 1;
}

/* n_sub flow sub-steps at the phi of the last compute_macros */
static void flow_substeps(orc_state* s) {
    const orc_params* p = &s->p;
    int N = s->N, nx = s->nx, ny = s->ny;
    {
        for (int sub = 0; sub < p->n_sub; ++sub) {
            fill_flow_walls(s, s->h, s->phi);
#pragma omp parallel for schedule(static)
            for (int x = 0; x < N; ++x) {
                double hx[9], post[9];
                for (int i = 0; i < 9; ++i) hx[i] = s->h[(size_t)i * N + x];
                collide_flow_node(p, s->L.L9, hx, s->phi[x], post, NULL);
                for (int i = 0; i < 9; ++i) s->ph[(size_t)i * N + x] = post[i];
            }
#pragma omp parallel for schedule(static)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    if (is_wall(s, x, y)) continue;
                    int d = y * nx + x;
                    for (int i = 0; i < 9; ++i) {
                        int src = wrap(y - C9Y[i], ny) * nx + wrap(x - C9X[i], nx);
                        s->hn[(size_t)i * N + d] = s->ph[(size_t)i * N + src];
                    }
                }
            swap_ptr(&s->h, &s->hn);
        }
    }
}

int orc_step(orc_state* s, long n) {
    if (n < 0) return -1;
    for (long i = 0; i < n; ++i) main_step(s);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Initialisation
 * ------------------------------------------------------------------------- */
int orc_set_fields(orc_state* s, const double* phi, const double* Cin, const double* thin,
                   const double* uxin, const double* uyin) {
    return orc_set_fields_ex(s, phi, Cin, thin, uxin, uyin, 0u);
}

/* The first moment of the phi populations that the local gradient scheme
 * (Sec. 3.1) maps back to a given gradient g:
 *   sum_i c_i f_i = -g/(3 s1) - W0^2 N(g)/tau0,
 * for g the isotropic D2Q9 central difference of the node field F,
 *   g = (1/cs^2) sum_i w_i c_i F(x + c_i)
 * (periodic wrap, or clamped at the channel walls). */
static void cd_first_moment(const orc_state* s, const double* F, int x, int y, double* V) {
    const orc_params* p = &s->p;
    double g[2];
    orc_stencil_gradient(p, F, x, y, g);
    double gx = g[0], gy = g[1];
    V[0] = V[1] = 0.0;
    if (gx * gx + gy * gy >= GRAD_GUARD) {
        double a, Nx, Ny;
        aniso_or_hook(p, gx, gy, &a, &Nx, &Ny);
        double s1 = s1_phi(p, a);
        double W2t = p->W0 * p->W0 / p->tau0;
        V[0] = -gx / (3.0 * s1) - W2t * Nx;
        V[1] = -gy / (3.0 * s1) - W2t * Ny;
    }
}

/* Melt velocity (main-step units) of the flow populations h9 at phi, as the
 * phi/C/theta update of a main step evaluates it (Sec. 3.4). */
static void main_step_velocity(const orc_state* s, const double* h9, double ph, double* u) {
    double us[2], Fb[2], uu[2], pr;
    flow_macros(&s->p, h9, ph, us, Fb, uu, &pr);
    u[0] = s->p.n_sub * uu[0];
    u[1] = s->p.n_sub * uu[1];
}

int orc_set_fields_ex(orc_state* s, const double* phi, const double* Cin, const double* thin,
                      const double* uxin, const double* uyin, unsigned flags) {
    const orc_params* p = &s->p;
    if (!phi) {
        set_err("phi is required");
        return -1;
    }
    if (flags & ~(ORC_KEEP_FLOW | ORC_KEEP_NONEQ)) {
        set_err("unknown flag");
        return -1;
    }
    int N = s->N, nx = s->nx, ny = s->ny;
    int keep_flow = (flags & ORC_KEEP_FLOW) && p->use_ns;
    int keep_neq = (flags & ORC_KEEP_NONEQ) != 0;
    int carry = keep_neq && s->hist_valid;
    /* the current fields (s->phi, C, U, H, theta, ux, uy; walls filled from
     * the inward node), read by the continuation flags; the loop below
     * writes populations and history only */
    if (flags) compute_macros(s);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int id = y * nx + x;
            double ph = phi[id];
            /* Reading: the phi populations carry the first moment that makes
             * the local gradient scheme reproduce the central-difference
             * gradient of phi. */
            double V[2], feq[5];
            cd_first_moment(s, phi, x, y, V);
            orc_eq_phi(ph, feq);
            if (keep_neq) {
                /* keep f - f^eq and the part of the first moment that the
                 * central difference does not explain */
                double Vo[2], fo_eq[5];
                cd_first_moment(s, s->phi, x, y, Vo);
                orc_eq_phi(s->phi[id], fo_eq);
                for (int i = 0; i < 5; ++i)
                    s->f[(size_t)i * N + id] += (feq[i] - fo_eq[i]) +
                                                3.0 * W5[i] * (C5X[i] * (V[0] - Vo[0]) + C5Y[i] * (V[1] - Vo[1]));
            } else {
                for (int i = 0; i < 5; ++i)
                    s->f[(size_t)i * N + id] = feq[i] + 3.0 * W5[i] * (C5X[i] * V[0] + C5Y[i] * V[1]);
            }

            double C;
            if (Cin) C = Cin[id];
            else if (p->c_init_U) C = 0.5 * (1.0 + p->k - (1.0 - p->k) * ph) * (1.0 + (1.0 - p->k) * p->U0);
            else C = p->C0;
            double th = thin ? thin[id] : p->theta0;
            double u[2] = {uxin ? uxin[id] : p->u_in_x, uyin ? uyin[id] : p->u_in_y};
            double h9[9];
            for (int i = 0; i < 9; ++i) h9[i] = s->h[(size_t)i * N + id];
            if (!p->use_ns) u[0] = u[1] = 0.0;
            if (keep_flow) main_step_velocity(s, h9, ph, u);
            double U = (2.0 * C / (1.0 + p->k - (1.0 - p->k) * ph) - 1.0) / (1.0 - p->k);
            double e5[5], o5[5];
            orc_eq_solute(C, ph, U, u[0], u[1], e5);
            if (keep_neq) {
                /* keep n - n^eq (Sec. 3.2) */
                orc_eq_solute(s->C[id], s->phi[id], s->U[id], s->ux[id], s->uy[id], o5);
                for (int i = 0; i < 5; ++i) s->n[(size_t)i * N + id] += e5[i] - o5[i];
            } else {
                for (int i = 0; i < 5; ++i) s->n[(size_t)i * N + id] = e5[i];
            }
            /* heat populations carry the velocity of their own time unit */
            const double ht = heat_sub(p);
            orc_eq_heat(th, ph, p->h_quintic, u[0] / ht, u[1] / ht, e5);
            if (keep_neq) {
                /* keep g - g^eq (Sec. 3.3) */
                orc_eq_heat(s->theta[id], s->phi[id], p->h_quintic, s->ux[id] / ht, s->uy[id] / ht, o5);
                for (int i = 0; i < 5; ++i) s->g[(size_t)i * N + id] += e5[i] - o5[i];
            } else {
                for (int i = 0; i < 5; ++i) s->g[(size_t)i * N + id] = e5[i];
            }
            double su[2] = {u[0], u[1]}; /* the velocity the next step evaluates */
            if (p->use_ns && !keep_flow) {
                double e9[9];
                orc_eq_flow(p->rho0, 0.0, u[0] / p->n_sub, u[1] / p->n_sub, e9);
                for (int i = 0; i < 9; ++i) s->h[(size_t)i * N + id] = e9[i];
                main_step_velocity(s, e9, ph, su);
            }
            /* time derivatives carry over at interior nodes:
             * history := new value - (current value - history) */
            int wall = p->walls && (x == 0 || y == 0 || x == nx - 1 || y == ny - 1);
            if (carry && !wall) {
                double pho = s->phi[id], omo = 1.0 - pho * pho;
                double Qo = pho * omo - p->lambda * (s->theta[id] + p->Mcinf * s->U[id]) * omo * omo;
                double om = 1.0 - ph * ph;
                double Q = ph * om - p->lambda * (th + p->Mcinf * U) * om * om;
                double H = th - 0.5 * h_of(ph, p->h_quintic);
                s->phi_prev[id] = ph - (pho - s->phi_prev[id]);
                s->Q_prev[id] = Q - (Qo - s->Q_prev[id]);
                if (p->use_ns) {
                    s->Cu_prev[id] = C * su[0] - (s->C[id] * s->ux[id] - s->Cu_prev[id]);
                    s->Cu_prev[N + id] = C * su[1] - (s->C[id] * s->uy[id] - s->Cu_prev[N + id]);
                    s->Hu_prev[id] = H * su[0] - (s->H[id] * s->ux[id] - s->Hu_prev[id]);
                    s->Hu_prev[N + id] = H * su[1] - (s->H[id] * s->uy[id] - s->Hu_prev[N + id]);
                }
            }
        }
    if (!keep_neq) s->hist_valid = 0;
    return 0;
}

int orc_init_seed(orc_state* s, const double* noise) {
    const orc_params* p = &s->p;
    int N = s->N;
    double* phi = alloc0(N);
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            double dx = x - p->seed_x, dy = y - p->seed_y;
            double d = sqrt(dx * dx + dy * dy);
            /* Sec. 4: phi = tanh[(R_s - d_s)/sqrt(2 W0)].  Reading: the
             * width is sqrt(2)*W0 (identical for W0 = 1). */
            double ph = tanh((p->seed_R - d) / (sqrt(2.0) * p->W0));
            if (noise && fabs(ph) < 0.9) ph += p->noise_amp * noise[y * s->nx + x];
            phi[y * s->nx + x] = ph;
        }
    int rc = orc_set_fields(s, phi, NULL, NULL, NULL, NULL);
    free(phi);
    return rc;
}

/* ---------------------------------------------------------------------------
 * Observation
 * ------------------------------------------------------------------------- */
int orc_get_fields(orc_state* s, double* out) {
    const orc_params* p = &s->p;
    int N = s->N;
    compute_macros(s);
    for (int x = 0; x < N; ++x) {
        out[x] = s->phi[x];
        out[N + x] = s->C[x];
        out[2 * N + x] = s->U[x];
        out[3 * N + x] = s->theta[x];
        out[4 * N + x] = s->ux[x];
        out[5 * N + x] = s->uy[x];
        double pr = 0.0;
        if (p->use_ns) {
            double hx[9], us[2], Fb[2], u[2];
            for (int i = 0; i < 9; ++i) hx[i] = s->h[(size_t)i * N + x];
            flow_macros(p, hx, s->phi[x], us, Fb, u, &pr);
            pr *= (double)p->n_sub * p->n_sub;
        }
        out[6 * N + x] = pr;
    }
    return 0;
}

int orc_get_pops(orc_state* s, int lattice, double* out) {
    int N = s->N;
    compute_macros(s);
    switch (lattice) {
        case 0: memcpy(out, s->f, sizeof(double) * 5 * N); return 0;
        case 1: memcpy(out, s->n, sizeof(double) * 5 * N); return 0;
        case 2: memcpy(out, s->g, sizeof(double) * 5 * N); return 0;
        case 3: memcpy(out, s->h, sizeof(double) * 9 * N); return 0;
    }
    return -1;
}

/* psi = atanh(phi), phi clamped to |phi| <= 1 - 2^-30.  Across a diffuse
 * interface of the model's tanh profile phi = tanh(d / (sqrt(2) W)), psi is
 * linear in the distance d, whatever the width and the direction. */
static double psi_of(double phi) {
    const double c = 1.0 - 1.0 / 1073741824.0;
    if (phi > c) phi = c;
    if (phi < -c) phi = -c;
    return atanh(phi);
}

/* Bilinear sample of psi from the four surrounding nodes; NaN outside
 * [0,nx-1] x [0,ny-1]. */
static double bilinear_psi(const orc_state* s, const double* F, double x, double y) {
    if (!(x >= 0.0 && y >= 0.0 && x <= s->nx - 1 && y <= s->ny - 1)) return NAN;
    int i0 = (int)floor(x), j0 = (int)floor(y);
    if (i0 > s->nx - 2) i0 = s->nx - 2;
    if (j0 > s->ny - 2) j0 = s->ny - 2;
    double fx = x - i0, fy = y - j0;
    const double* r0 = F + (size_t)j0 * s->nx;
    const double* r1 = r0 + s->nx;
    return (1.0 - fx) * (1.0 - fy) * psi_of(r0[i0]) + fx * (1.0 - fy) * psi_of(r0[i0 + 1]) +
           (1.0 - fx) * fy * psi_of(r1[i0]) + fx * fy * psi_of(r1[i0 + 1]);
}

/* Reading of the tip measurement (the paper's tip plots are not recoverable):
 * arm k points along angle orient + k pi/2 from the seed centre.  psi =
 * atanh(phi) is sampled every 1 lu along the ray (bilinear in psi); the tip
 * is the outermost sample pair with psi_j > 0 >= psi_{j+1}, refined
 * linearly in psi:
 *   s = j + psi_j / (psi_j - psi_{j+1}),
 * which is exact for a planar tanh interface of any width and orientation
 * (interpolating phi itself would add a sub-lattice error that oscillates as
 * the tip crosses nodes).  The tip radius fits s(w) = s0 - w^2/(2 rho) by
 * least squares over rays shifted sideways by w = -3..3. */
static double ray_crossing(const orc_state* s, int k, double w) {
    const orc_params* p = &s->p;
    double th = p->orient + k * (M_PI / 2.0);
    double dx = cos(th), dy = sin(th), ex = -sin(th), ey = cos(th);
    double best = NAN;
    double prev = NAN;
    for (int j = 0;; ++j) {
        double x = p->seed_x + j * dx + w * ex, y = p->seed_y + j * dy + w * ey;
        double v = bilinear_psi(s, s->phi, x, y);
        if (isnan(v)) break;
        if (j > 0 && prev > 0.0 && v <= 0.0) best = (j - 1) + prev / (prev - v);
        prev = v;
    }
    return best;
}

static double tip_radius(const orc_state* s, int k) {
    double Sx = 0, Sy = 0, Sxx = 0, Sxy = 0;
    int n = 0;
    for (int w = -3; w <= 3; ++w) {
        double c = ray_crossing(s, k, (double)w);
        if (isnan(c)) continue;
        double X = (double)(w * w);
        Sx += X;
        Sy += c;
        Sxx += X * X;
        Sxy += X * c;
        ++n;
    }
    if (n < 3) return NAN;
    double den = n * Sxx - Sx * Sx;
    if (den == 0.0) return NAN;
    double B = (n * Sxy - Sx * Sy) / den;
    if (!(B < 0.0)) return NAN;
    return -1.0 / (2.0 * B);
}

int orc_reduce(orc_state* s, double* out) {
    const orc_params* p = &s->p;
    int N = s->N;
    compute_macros(s);
    double sC = 0, sH = 0, sphi = 0, bad = 0, Fx = 0, Fy = 0, cx = 0, cy = 0;
    for (int x = 0; x < N; ++x) {
        sC += s->C[x];
        sH += s->H[x];
        double w = 0.5 * (1.0 + s->phi[x]);
        sphi += w;
        cx += w * (x % s->nx);
        cy += w * (x / s->nx);
        int ok = isfinite(s->phi[x]) && isfinite(s->C[x]) && isfinite(s->H[x]);
        if (p->use_ns) ok = ok && isfinite(s->ux[x]) && isfinite(s->uy[x]);
        if (!ok) bad += 1;
    }
    cx /= sphi;
    cy /= sphi;
    double T = 0, Fsx = 0, Fsy = 0;
    if (p->use_ns) {
        /* Eq. (hydrodynamic force/torque), reading: summed over all nodes of
         * the force actually applied, [1 - q(phi)] f, sub-step units; the
         * literal form, f summed over the nodes covered by the solid
         * (phi > 0), is reported as well.  f = (u_s - u*)/dt' with u_s = 0. */
        for (int x = 0; x < N; ++x) {
            double hx[9], us[2], Fb[2], u[2], pr;
            for (int i = 0; i < 9; ++i) hx[i] = s->h[(size_t)i * N + x];
            flow_macros(p, hx, s->phi[x], us, Fb, u, &pr);
            Fx -= Fb[0];
            Fy -= Fb[1];
            double rx = (x % s->nx) - cx, ry = (x / s->nx) - cy;
            T -= rx * Fb[1] - ry * Fb[0];
            if (s->phi[x] > 0.0) {
                Fsx += us[0]; /* -f = u* */
                Fsy += us[1];
            }
        }
    }
    out[0] = sC;
    out[1] = sH;
    out[2] = sphi / N;
    out[3] = bad;
    out[4] = Fx;
    out[5] = Fy;
    out[6] = T;
    for (int k = 0; k < 4; ++k) {
        out[7 + k] = ray_crossing(s, k, 0.0);
        out[11 + k] = tip_radius(s, k);
    }
    out[15] = cx;
    out[16] = cy;
    out[17] = Fsx;
    out[18] = Fsy;
    return 0;
}
