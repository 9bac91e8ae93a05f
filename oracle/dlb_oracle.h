/*
 * dlb_oracle.h -- CPU FP64 reference ("oracle") for the diffuse-interface
 * multi-relaxation-time lattice Boltzmann method of Zhan, Chai, Shi, Jiang,
 * Geng and Sun, "A diffuse-interface lattice Boltzmann method for the
 * dendritic growth with thermosolutal convection" (arXiv:2209.01444).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark, never by the
 * product path.  It shares no code, header, table or helper with the GPU
 * library; the two meet only in the tests, which feed both the same seeded
 * inputs.
 *
 * Units: lattice units, dx = 1, main step dt = 1, c = 1, cs^2 = 1/3
 * (Appendix B).  The flow lattice runs N_sub sub-steps of dt' = dt/N_sub per
 * main step (two-time-scaling, Sec. 4 preamble); inside it velocities are in
 * lattice units per sub-step.  Everything this header returns is in main-step
 * units unless stated otherwise.
 *
 * Parity status of each part (how it is pinned; see tests/test_oracle_*.py):
 *   D2Q5/D2Q9 transforms, Lambda, equilibria, forcing moments   pinned
 *   anisotropy a_s and N                                          pinned
 *   phi lattice: modified streaming, source, local gradient       pinned
 *   solute / heat lattices: diffusion, conservation, d_t(Cu)      pinned
 *   flow lattice: viscosity, diffuse solid forcing                pinned
 *   anti-trapping current J_at: no printed number isolates it; the GPU
 *     path matches this one in isothermal alloy runs and its dendrite
 *     freezes the Gibbs-Thomson concentration of Sec. 4.3 into the
 *     solid within 0.3% (18% off without J_at)                    indirect
 *   non-equilibrium-extrapolation walls: uniform channel flow steady (pinned);
 *     beyond it only through the GPU path it matches to 1e-10, whose
 *     stationary-cylinder drag is within 3.2% of the values printed in
 *     the table of Sec. 4.1                                       indirect
 *   restart flags (orc_set_fields_ex): continuation is exact      pinned
 *   stencil-gradient ablation (grad_stencil): exact on quadratics,
 *     stationary planar fronts at second order                    pinned
 *   heat sub-steps (n_sub_t): diffusion rate, advected mode       pinned
 *   external force F with varphi: population forcing against the
 *     printed moment vector; uniform acceleration exact; force-driven
 *     channel flow against the parabola; uniform pressure across it   pinned
 *   far-field walls (walls = 2): sine modes vanishing on the wall
 *     ring decay at the diffusion rate; relaxation to the far field pinned
 *   tip position / radius measurement                             pinned (geometry)
 */
#ifndef DLB_ORACLE_H
#define DLB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
    int nx, ny;
    int use_c;        /* solute lattice on (else U = U0 everywhere)          */
    int use_t;        /* heat lattice on (else theta = theta0 everywhere)     */
    int use_ns;       /* flow lattice on (else u = 0)                         */
    int walls;        /* 0: periodic; 1: channel (west inflow, east outflow,
                         free-slip north/south, zero-gradient phi/C/H);
                         2: far field (Sec. 4.4): the wall ring holds phi = -1,
                         the initial far-field C and theta0 by extrapolation;
                         flow lattice off, local gradient, one heat step    */
    int n_sub;        /* flow sub-steps per main step (two-time-scaling N)    */
    int h_quintic;    /* 0: h(phi)=phi; 1: h = 15(phi-2phi^3/3+phi^5/5)/8    */
    int c_init_U;     /* 0: initial C uniform = C0; 1: initial U uniform = U0 */
    int grad_max_iter;/* cap on the implicit local-gradient iteration         */
    int phi_static;   /* 1: phi, C and theta stay as set; only the flow lattice
                         steps (n_sub sub-steps per main step) past the frozen
                         diffuse solid: the stationary-cylinder problem      */
    int grad_stencil; /* 0: the local gradient of Sec. 3.1 (the method);
                         1: ablation, grad phi from the isotropic nine-point
                         difference of the node values of phi               */
    int n_sub_t;      /* heat sub-steps per main step (multi-time-scaling for
                         Le = alpha/D != 1); 0 or 1: one                      */
    double W0, tau0, eps4, orient, lambda, Mcinf, k, D, alpha, nu, rho0;
    double u_in_x, u_in_y;   /* inflow / initial velocity, lu per main step  */
    double theta0, U0, C0;
    double seed_R, seed_x, seed_y, noise_amp;
    double grad_tol;  /* relative stopping tolerance of the gradient iteration*/
    double fixed_as;  /* test hook: >0 fixes a_s to this value and N to 0     */
    double force_x, force_y; /* external body force F (Sec. 3.4), lu per main
                         step^2; the flow sub-steps take F / N_sub^2          */
    double varphi;    /* adjustable parameter of the forcing (Sec. 3.4); the
                         paper's runs use 0                                    */
} orc_params;

typedef struct orc_state orc_state;

/* Lifecycle.  orc_create returns NULL when a relaxation rate leaves (0,2) or
 * the grid is smaller than 3x3. */
orc_state* orc_create(const orc_params* p);
void       orc_destroy(orc_state* s);
const char* orc_last_error(void);

/* Initial condition of Sec. 4: diffuse circular seed
 *   phi = tanh[(R_s - d_s)/(sqrt(2) W0)]
 * plus noise_amp*noise[x] where |phi| < 0.9 (noise: nx*ny host doubles, or
 * NULL).  Then orc_set_fields semantics. */
int orc_init_seed(orc_state* s, const double* noise);

/* Re-initialise every lattice to equilibrium at the given macroscopic fields
 * (each nx*ny, row-major y*nx+x; NULL -> parameter default: C from C0/U0,
 * theta0, u_in).  The phi populations also carry the first moment that makes
 * the local gradient scheme return the central-difference gradient of phi.
 * History is reset (time derivatives are zero on the next step).  p := 0. */
int orc_set_fields(orc_state* s, const double* phi, const double* C,
                   const double* theta, const double* ux, const double* uy);

/* orc_set_fields with continuation flags, for restarting from fields that
 * were advanced outside the lattice Boltzmann method:
 *   ORC_KEEP_FLOW:  the flow lattice keeps its populations; the C and theta
 *                   equilibria use the velocity of the current flow state
 *                   (ux, uy ignored).
 *   ORC_KEEP_NONEQ: the solute and heat lattices keep their non-equilibrium
 *                   parts: each population moves by the change of its
 *                   equilibrium between the current and the new fields.
 * The phi lattice and the history are set as by orc_set_fields. */
#define ORC_KEEP_FLOW 1u
#define ORC_KEEP_NONEQ 2u
int orc_set_fields_ex(orc_state* s, const double* phi, const double* C,
                      const double* theta, const double* ux, const double* uy,
                      unsigned flags);

int  orc_step(orc_state* s, long nsteps);
long orc_step_count(const orc_state* s);

/* Seven planes of nx*ny: phi, C, U, theta, ux, uy (lu/main step), p
 * (main-step units). */
int orc_get_fields(orc_state* s, double* out);

/* Raw populations of one lattice (0 phi, 1 C, 2 H, 3 flow), q*nx*ny,
 * pre-collision at the current step; flow slot 0 unshifted (includes rho0). */
int orc_get_pops(orc_state* s, int lattice, double* out);

/* Reductions, out[0..18]:
 *   0 sum C, 1 sum H, 2 solid fraction sum((1+phi)/2)/N, 3 non-finite count,
 *   4,5 hydrodynamic force Fx,Fy = -sum [1-q(phi)] f, 6 torque (flow
 *   sub-step units), 7..10 tip position s_k of arms k=0..3, 11..14 tip
 *   radius rho_k, 15,16 solid centroid, 17,18 force -sum f over the nodes
 *   with phi > 0 */
int orc_reduce(orc_state* s, double* out);

/* ---- single-node primitives, exposed for the pins ---- */
void orc_m_d2q5(double* M25);
void orc_m_d2q9(double* M81);
void orc_lambda_d2q5(double s0, double s1, double s2, double* L25);
void orc_lambda_d2q9(const double* s9, double* L81);
void orc_eq_phi(double phi, double* out5);
void orc_eq_solute(double C, double phi, double U, double ux, double uy, double* out5);
void orc_eq_heat(double theta, double phi, int h_quintic, double ux, double uy, double* out5);
void orc_eq_flow(double rho0, double p, double ux, double uy, double* out9);
void orc_force_flow(double Fx, double Fy, double* out9);
/* The full forcing populations of Sec. 3.4: the first-order part carries
 * G = F + [1 - q] f, the varphi part (uF + Fu):(cc - cs^2 I)/(2 cs^4) the
 * external force F and the velocity u. */
void orc_force_flow_full(double Gx, double Gy, double Fx, double Fy, double ux, double uy,
                         double varphi, double* out9);
void orc_anisotropy(double eps4, double orient, double gx, double gy, double* out3);
/* out: gx, gy, a_s, Nx, Ny, iterations */
void orc_local_gradient(const orc_params* p, double m1x, double m1y, double* out6);
/* Stencil gradient at node (x, y) of the node field phi (nx*ny): the
 * isotropic difference 3 sum_i w_i c_i phi(x + c_i) with the D2Q9 weights
 * (periodic wrap, or clamped at the channel walls); out: gx, gy. */
void orc_stencil_gradient(const orc_params* p, const double* phi, int x, int y, double* out2);
/* One flow collision at a node (sub-step units): pre-collision h (9, slot 0
 * unshifted), frozen phi -> post-collision populations; aux[0..3] = u*, u. */
void orc_collide_flow(const orc_params* p, const double* h, double phi,
                      double* post, double* aux);

#ifdef __cplusplus
}
#endif
#endif
