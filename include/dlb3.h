/*
 * dlb3.h -- C ABI of the three-dimensional phase-field, solute and heat
 * lattices (D3Q7) of the diffuse-interface lattice Boltzmann method of
 * Zhan et al., arXiv:2209.01444 (Sec. 2 anisotropy a_s and N for any d,
 * Secs. 3.1-3.3 with a general lattice sound speed), and optionally the melt
 * flow of Sec. 3.4 on D3Q19 (periodic, or a channel with walls).
 * Exported by libdlb.so beside the 2-D solver (dlb.h).
 *
 * Lattice: c0 = 0, c1..c3 = +x, +y, +z, c4..c6 = -x, -y, -z; cs^2 = 1/4,
 * w0 = 1/4, w1..6 = 1/8; S = diag(1, s1, s1, s1, 1, 1, 1) for each lattice.
 * Crystal axes along the lattice axes.  One main step: every lattice reads
 * the fields of time t (Jacobi), phi with the modified streaming of Sec. 3.1.
 * Melt flow (use_ns): D3Q19 (c0, six faces, twelve edges; w = 1/3, 1/18,
 * 1/36; cs^2 = 1/3), equilibrium, pressure and diffuse force of Sec. 3.4
 * (varphi = 0), MRT with s2 = 1/(3 nu/n_sub + 1/2) on the six second moments
 * and 1 on the rest; n_sub sub-steps per main step at the frozen phi of time
 * t; the solute and heat equilibria take u = n_sub u'.
 *
 * Ownership: the caller owns the device state buffer (dlb3_state_bytes) and
 * the stream; the library owns only the small host handle.  dlb3_step and
 * dlb3_init_seed are asynchronous on the stream; dlb3_set_fields (which
 * copies the caller's host arrays), dlb3_get_fields and dlb3_reduce
 * synchronise it before they return.  Calls on one handle must not overlap.
 * Errors: 0 on success; a negative DLB3_E* code otherwise, with a message
 * for dlb3_last_error().  No C++ exception crosses the ABI.
 */
#ifndef DLB3_H
#define DLB3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { DLB3_OK = 0, DLB3_EINVAL = -1, DLB3_ENOMEM = -2, DLB3_EHIP = -3 };
/* Population storage / arithmetic type. */
enum {
    DLB3_F64 = 0,  /* FP64 storage, arithmetic and history                        */
    DLB3_F32 = 1,  /* FP32 storage, arithmetic and history                        */
    DLB3_F16S = 2, /* FP16 storage of each D3Q7 population's difference from its
                      value in the initial far-field liquid at rest (phi = -1, C
                      and theta as initialised, moving at u0 with melt flow) and
                      of the D3Q19 populations (h_0 - rho0); FP32 arithmetic and
                      history; FP64 reductions and field output                 */
    DLB3_BF16S = 3 /* as DLB3_F16S with BF16 storage                              */
};

typedef struct dlb3_params {
    int32_t nx, ny, nz;   /* grid, >= 8 each                                     */
    int32_t walls;        /* 0 periodic; 1 zero-gradient walls (outermost layer
                             of nodes rebuilt as a copy of the inward neighbour) */
    int32_t use_t;        /* 1 heat lattice; 0 isothermal (theta = theta0)       */
    int32_t h_quintic;    /* h(phi): 0 phi; 1 15(phi - 2phi^3/3 + phi^5/5)/8     */
    int32_t c_init_U;     /* initial solute: 0 uniform C0; 1 uniform U0          */
    int32_t precision;    /* DLB3_F64, DLB3_F32, DLB3_F16S or DLB3_BF16S         */
    int32_t grad_iters;   /* cap of the local-gradient fixed point (0: default)  */
    double W0, tau0, eps4;       /* interface width, kinetic time, anisotropy    */
    double lambda, Mcinf, k;     /* coupling, M c_inf, partition coefficient     */
    double D, alpha;             /* solute and heat diffusivities (lu^2/step)    */
    double theta0, U0, C0;       /* initial temperature, supersaturation, C      */
    double seed_R, seed_x, seed_y, seed_z; /* spherical seed (lu, node coords)   */
    double grad_tol;             /* tolerance of the gradient fixed point (0: default) */
    int32_t use_ns;              /* 1: melt flow; with walls the channel: west inlet
                                    u0, east outflow (p = 0), free slip on the y and
                                    z faces, by non-equilibrium extrapolation      */
    int32_t n_sub;               /* flow sub-steps per main step (two-time-scaling) */
    double nu, rho0;             /* viscosity (lu^2 per main step), density       */
    double u0[3];                /* initial velocity (lu per main step); the Mach
                                    number |u0| sqrt(3)/n_sub must stay below 0.3 */
} dlb3_params;

typedef struct dlb3_solver* dlb3_handle;

/* Bytes of device state for p (populations, history, a staging area of
 * eight double planes); 0 if p is invalid (message in dlb3_last_error). */
size_t dlb3_state_bytes(const dlb3_params* p);

/* Bind a solver to a caller-owned device buffer of at least
 * dlb3_state_bytes(p) bytes and a hipStream_t (NULL: the null stream). */
int dlb3_create(const dlb3_params* p, void* dev_state, size_t bytes, void* hip_stream, dlb3_handle* out);
int dlb3_destroy(dlb3_handle h);

/* Initial condition of Sec. 4 in 3-D: phi = tanh[(R - d)/(sqrt(2) W0)] about
 * the seed centre, C from C0 or U0, theta0; then dlb3_set_fields. */
int dlb3_init_seed(dlb3_handle h);

/* Every lattice at equilibrium at the given fields (host arrays of nx*ny*nz
 * doubles, x fastest then y then z; C, theta and the velocity components
 * nullable: defaults from the parameters), the phi populations with the first
 * moment that makes the local scheme return the isotropic D3Q19 central
 * difference of phi; the flow at p = 0 and u' = u/n_sub.  The history is
 * reset (time derivatives zero on the next step). */
int dlb3_set_fields(dlb3_handle h, const double* phi, const double* C, const double* theta, const double* ux,
                    const double* uy, const double* uz);

/* n >= 0 main steps. */
int dlb3_step(dlb3_handle h, int64_t n);

/* phi, C, U, theta, ux, uy, uz (lu per main step; 0 without flow) and p
 * (main-step units) into host out (8 planes of nx*ny*nz doubles). */
int dlb3_get_fields(dlb3_handle h, double* out);

/* out[0..9]: sum C, sum H, solid fraction sum((1 + phi)/2)/N, non-finite
 * count, tip distance from the seed node (centre rounded to the nearest node)
 * along +x, +y, +z, -x, -y, -z (last + to - crossing of phi on the axis,
 * refined linearly in atanh(phi); -1 if none). */
int dlb3_reduce(dlb3_handle h, double* out);

const char* dlb3_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
