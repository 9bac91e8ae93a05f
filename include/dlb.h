/*
 * dlb.h -- C ABI of libdlb.so, the MI355X (gfx950) solver for the
 * diffuse-interface multi-relaxation-time lattice Boltzmann method of
 * Zhan, Chai, Shi, Jiang, Geng and Sun, "A diffuse-interface lattice
 * Boltzmann method for the dendritic growth with thermosolutal convection"
 * (arXiv:2209.01444).
 *
 * The statement of the problem is the paper's: the phase field phi of the
 * anisotropic phase-field equation (Sec. 2, Sec. 3.1, D2Q5), the solute C and
 * supersaturation U (Sec. 3.2, D2Q5), the heat variable H and temperature
 * theta (Sec. 3.3, D2Q5), and the melt flow u, p with the order-parameter
 * fluid-solid force [1 - q(phi)] f (Sec. 3.4, D2Q9), advanced together by
 * dt; the flow lattice takes N_sub sub-steps of dt/N_sub (two-time-scaling,
 * Sec. 4 preamble).
 *
 * Units are lattice units: dx = 1, main step dt = 1, c = 1, cs^2 = 1/3.
 * Velocities are in lu per main step, pressure in main-step units.
 * Fields are row-major nx*ny planes, index y*nx + x.
 *
 * Memory: the caller owns the device state buffer (dev_state, at least
 * dlb_state_bytes bytes, 256-byte aligned) and the HIP stream; the library
 * owns only the small host-side handle.  All calls are asynchronous on the
 * stream unless they say otherwise.  No C++ exception crosses this ABI.
 *
 * Errors: every int-returning call returns DLB_OK (0) or a negative code;
 * dlb_last_error() describes the last failure of the calling thread.
 */
#ifndef DLB_H
#define DLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DLB_OK = 0,
    DLB_EINVAL = -1,      /* bad argument: relaxation rate outside (0,2), grid < 16x16,
                             unknown precision, null handle, n < 0 ...              */
    DLB_ENOMEM = -2,      /* state buffer smaller than dlb_state_bytes()          */
    DLB_EHIP = -3,        /* a HIP call failed; dlb_last_error() has its message  */
    DLB_ENAN = -4,        /* a reduction found non-finite values                  */
    DLB_EUNSUPPORTED = -5 /* combination not built                                */
};

/* Population storage / compute precision. */
enum {
    DLB_F64 = 0,   /* FP64 storage and arithmetic                                  */
    DLB_F32 = 1,   /* FP32 storage and history; FP32 arithmetic in the flow
                      sub-steps, FP64 arithmetic in the phi/C/theta step (the
                      supersaturation U magnifies its rounding in the solid)      */
    DLB_F16S = 2,  /* FP16 storage of shifts from the rest-state populations,
                      FP32 arithmetic and history, FP64 reductions                 */
    DLB_BF16S = 3, /* as DLB_F16S with BF16 storage                                */
    DLB_F32M = 4,  /* FP32 storage and history, FP64 arithmetic everywhere          */
    DLB_F16SM = 5  /* mixed: the phi and flow populations as FP16 shifts from the
                      rest state, the solute and heat populations in FP32; FP32
                      history and flow arithmetic, FP64 arithmetic in the
                      phi/C/theta step, FP64 reductions                           */
};

/* Boundary configuration. */
enum {
    DLB_BC_PERIODIC = 0,
    /* Channel (Sec. 4.2, non-equilibrium extrapolation of Sec. 4 preamble):
     * the outermost ring of nodes are wall nodes whose populations are
     * rebuilt from the inward neighbour x_f (diagonal at corners) whenever
     * they are read:  f(x_b) = f^eq(Psi_b, u_b) + f(x_f) - f^eq(Psi_f, u_f).
     * phi, C, H: zero gradient (a copy of x_f).  Flow: west x=0 inflow
     * u_b = u_in, p_b = p_f; east x=nx-1 du/dx = 0 with p_b = 0 (u_b,y = 0 at
     * its corners); north/south free slip u_b = (u_f,x, 0), p_b = p_f. */
    DLB_BC_CHANNEL = 1,
    /* Far field (Sec. 4.4: Dirichlet phi = -1, U = U0, theta = theta0 on the
     * outer boundary): the outermost ring are wall nodes as in the channel;
     * their phi, C and H populations are rebuilt toward the far-field liquid,
     *   f(x_b) = f^eq(Psi_inf, 0) + f(x_f) - f^eq(Psi_f, 0),
     * Psi_inf = (phi = -1, C of the initial far field, theta0), u = 0.
     * Requires use_ns = 0, grad_stencil = 0, n_sub_t <= 1 and phi_static = 0
     * (DLB_EUNSUPPORTED otherwise); not available in batches. */
    DLB_BC_FARFIELD = 2
};

typedef struct dlb_params {
    int32_t nx, ny;       /* grid, >= 16 each                                       */
    int32_t use_ns;       /* 1: flow lattice on; 0: u = 0 (phi, C, theta always on)  */
    int32_t bc;           /* DLB_BC_*                                                */
    int32_t n_sub;        /* flow sub-steps per main step (Sec. 4: N = 15)           */
    int32_t h_quintic;    /* 0: h(phi) = phi; 1: 15(phi - 2phi^3/3 + phi^5/5)/8      */
    int32_t c_init_U;     /* initial solute: 0 uniform C = C0; 1 uniform U = U0      */
    int32_t precision;    /* DLB_F64 .. DLB_F16SM                                    */
    int32_t grad_iters;   /* cap of the local-gradient fixed point (0: default)      */
    int32_t flow_fuse;    /* flow sub-steps fused per launch: 1, 3 or 5 (0: 5 with
                             FP32 flow arithmetic, 3 with FP64: f64, f32m); the
                             fused kernel keeps a tile in registers and LDS for
                             that many sub-steps; results equal the unfused ones */
    int32_t phi_static;   /* 1: phi, C and theta stay as set (no phi/C/theta
                             update); each main step is n_sub flow sub-steps past
                             the frozen diffuse solid -- the stationary-cylinder
                             problem of Sec. 4.1.  Not available in batches     */
    int32_t isothermal;   /* 1: theta = theta0 everywhere, no heat lattice (the
                             isothermal alloy of Sec. 4.3)                       */
    int32_t grad_stencil; /* 0: grad phi by the local scheme of Sec. 3.1 (the
                             method); 1: ablation, grad phi from the isotropic
                             nine-point difference of the node values of phi
                             (one extra plane in the state).  Not available in
                             batches                                             */
    int32_t n_sub_t;      /* heat sub-steps per main step (multi-time-scaling for
                             a Lewis number alpha/D != 1): the heat lattice takes
                             n_sub_t steps of dt/n_sub_t with phi frozen at its
                             time-t value, diffusivity alpha/n_sub_t per
                             sub-step.  0 or 1: one step inside the phi/C/theta
                             update.  Not available in batches                   */
    int32_t tile_rows;    /* rows of the fused flow tile (FP32 flow arithmetic,
                             flow_fuse 3 or 5): 32 (8 waves) or 48 (12 waves:
                             less halo, fewer tiles resident); 0 chooses 48
                             where the grid has at least four rounds of tall
                             tiles for the device's compute units, else 32.
                             Results do not depend on it.  48 with FP64 flow
                             arithmetic or unfused sub-steps: DLB_EUNSUPPORTED.
                             Batches use 32                                      */
    double W0, tau0;      /* interface width and kinetic time (Sec. 2)              */
    double eps4, orient;  /* anisotropy strength and crystal orientation (rad)      */
    double lambda, Mcinf, k;   /* coupling, M c_inf, partition coefficient          */
    double D, alpha, nu;  /* solute and heat diffusivities, viscosity (main units)  */
    double rho0;          /* constant density of the flow model (Sec. 3.4)          */
    double u_in_x, u_in_y;/* inflow / initial velocity                              */
    double theta0, U0, C0;/* initial temperature, supersaturation, concentration    */
    double seed_R, seed_x, seed_y; /* seed radius and centre (lu, node coordinates)  */
    double noise_amp;     /* amplitude applied to the caller's noise field          */
    double grad_tol;      /* relative tolerance of the gradient fixed point (0: default) */
    double force_x, force_y; /* external body force F of Sec. 3.4 (lu per main
                             step^2; the flow sub-steps take F/n_sub^2); needs
                             use_ns = 1 and flow_fuse 0 or 1 (each sub-step is
                             one launch); not available in batches             */
    double varphi;        /* adjustable parameter of the forcing (Sec. 3.4): the
                             second-order force terms (uF + Fu) and the pressure
                             term varphi K u.F with K = 2(s2 - 3 s4 + s2 s4) /
                             (9 s2 s4), s4 = 1; the paper's runs use 0         */
} dlb_params;

typedef struct dlb_solver* dlb_handle;

/* Bytes of device state needed for p; 0 if p is invalid. Pure. */
size_t dlb_state_bytes(const dlb_params* p);

/* Bind a solver to a caller-owned device buffer and stream (hipStream_t, may
 * be NULL for the null stream).  Nothing is initialised on the device. */
int dlb_create(const dlb_params* p, void* dev_state, size_t bytes, void* hip_stream,
               dlb_handle* out);
int dlb_destroy(dlb_handle h);

/* Initial condition of Sec. 4: the diffuse seed
 *   phi = tanh[(R_s - d_s)/(sqrt(2) W0)]
 * centred at (seed_x, seed_y), plus noise_amp * noise[x] where |phi| < 0.9
 * (noise: nx*ny doubles on the host, or NULL); then as dlb_set_fields with
 * the parameter defaults.  Synchronises the stream. */
int dlb_init_seed(dlb_handle h, const double* noise);

/* Re-initialise every lattice at the given macroscopic fields (nx*ny doubles
 * each; phi required, others NULL for the parameter default: C from C0/U0,
 * theta0, u_in).  Populations are set to their equilibria (Sec. 3.1-3.4,
 * p = 0); the phi populations also carry the first moment that makes the
 * local gradient of Sec. 3.1 return the isotropic central-difference
 * gradient of phi.  Time derivatives restart from zero.  on_device: 1 if the
 * pointers are device memory.  Synchronises the stream when on_device = 0. */
int dlb_set_fields(dlb_handle h, const double* phi, const double* C, const double* theta,
                   const double* ux, const double* uy, int on_device);

/* dlb_set_fields with continuation flags, for restarting from fields that
 * were advanced outside the lattice Boltzmann method (a learned jump):
 *   DLB_KEEP_FLOW:  the flow lattice keeps its populations; the C and theta
 *                   equilibria use its velocity at the new phi (ux, uy are
 *                   ignored).
 *   DLB_KEEP_NONEQ: the phi, C and H populations keep their non-equilibrium
 *                   parts: each moves by the change of its equilibrium
 *                   (Sec. 3.1-3.3) between the current and the new fields,
 *                   and the phi first moment also by the change of its
 *                   central-difference gradient term; at interior nodes the
 *                   time derivatives of phi, Q, Cu and Hu carry over
 *                   (history := new value - (current value - history)).
 * With both flags, restarting at the state's own fields changes nothing
 * beyond rounding.  KEEP_NONEQ uses the idle ping-pong population buffer as
 * scratch.  Unknown flag bits: DLB_EINVAL. */
#define DLB_KEEP_FLOW 1u
#define DLB_KEEP_NONEQ 2u
int dlb_set_fields_ex(dlb_handle h, const double* phi, const double* C, const double* theta,
                      const double* ux, const double* uy, int on_device, uint32_t flags);

/* Advance n >= 0 main steps (asynchronous). */
int dlb_step(dlb_handle h, int64_t n);

/* As dlb_step (without graph replay), recording HIP events on the solver's
 * stream before and after the phi/C/theta kernel and after the last flow
 * launch of every main step; returns the summed milliseconds of the
 * phi/C/theta kernels and of the back-to-back flow launches, and the
 * number of launches of each (a fused launch counts once).  Synchronises the
 * stream after every step. */
int dlb_step_timed(dlb_handle h, int64_t n, double* ms_pct, double* ms_flow,
                   int64_t* launches_pct, int64_t* launches_flow);

int64_t dlb_step_count(dlb_handle h);

/* Macroscopic fields (Sec. 3.1-3.4) at the current step.  mask bit f selects
 * field f of (phi, C, U, theta, ux, uy, p); out receives the selected fields
 * in that order, nx*ny each, as doubles (out_f32 = 0) or floats.
 * out_on_device: 1 if out is device memory (asynchronous), else the call
 * synchronises. */
int dlb_get_fields(dlb_handle h, uint32_t mask, void* out, int out_on_device, int out_f32);

/* dlb_get_fields for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same fields, mask and layout as dlb_get_fields with out_on_device = 0,
 * staged through a static device buffer of DLB_NOALLOC_SCRATCH_BYTES that
 * each GPU holds from the first call until the process ends; no hipMalloc,
 * hipFree or other allocating call.  out is host memory of
 * popcount(mask) * nx * ny values (doubles, or floats with out_f32 = 1),
 * owned by the caller.  Synchronises the solver's stream.
 * Errors: DLB_EINVAL for a null handle or output, a bad mask, or a selection
 * larger than DLB_NOALLOC_SCRATCH_BYTES (use dlb_get_fields); DLB_EHIP.
 * All calls on one GPU share its buffer: calls that overlap on one GPU (from
 * several host threads) race. */
#define DLB_NOALLOC_SCRATCH_BYTES (32u << 20)
int dlb_get_fields_noalloc(dlb_handle h, uint32_t mask, void* out, int out_f32);

/* Reductions in FP64 on the device; synchronises.  out[0..18] (19 doubles):
 *   0 sum C, 1 sum H, 2 solid fraction sum((1+phi)/2)/(nx ny), 3 non-finite
 *   count, 4-5 hydrodynamic force (Sec. 3.4) -sum [1-q(phi)] f over all nodes,
 *   6 torque about the solid centroid (flow sub-step units), 7-10 tip
 *   position s_k of arm k (angle orient + k pi/2 from the seed centre), 11-14
 *   tip radius rho_k, 15-16 solid centroid, 17-18 the force in the literal
 *   form of Sec. 3.4, -sum f over the nodes covered by the solid (phi > 0),
 *   f = -u* (u_s = 0, sub-step units).
 * Tip: psi = atanh(phi) (phi clamped to |phi| <= 1 - 2^-30) sampled every
 * 1 lu along the arm ray by bilinear interpolation of the node values of
 * psi; s is the outermost sample pair psi_j > 0 >= psi_{j+1}, refined
 * linearly in psi (exact for a planar tanh interface at any orientation);
 * rho fits s(w) = s0 - w^2/(2 rho) over rays offset sideways by w = -3..3.
 * Returns DLB_ENAN when the non-finite count is positive (out still filled). */
int dlb_reduce(dlb_handle h, double* out);

/* Checkpoint: the whole device state plus step counter and history flag.
 * dlb_checkpoint_bytes() gives the host buffer size.  Synchronise. */
size_t dlb_checkpoint_bytes(dlb_handle h);
int dlb_save(dlb_handle h, void* host_buf, size_t bytes);
int dlb_load(dlb_handle h, const void* host_buf, size_t bytes);

/* Copy the whole state (device buffer and step counter) of src into dst,
 * device to device; both solvers must have identical parameters.  Ordered
 * on src's stream (and waits for it when the streams differ). */
int dlb_copy_state(dlb_handle dst, dlb_handle src);

int dlb_sync(dlb_handle h);

/* FP64 equilibria of the four lattices evaluated on the device by the same
 * functions the initialisation and the walls use (Sec. 3.1-3.4), for n
 * host tuples macros[8*i..] = (phi, C, U, theta, ux, uy, p, rho0);
 * out[24*i..] = f^eq(5), n^eq(5), g^eq(5), h^eq(9).  Evaluation order (no
 * contraction): f_i = w_i*phi; q = 0.5*(1-phi), qU = q*U, n_0 = C +
 * (w_0-1)*qU, n_i = w_i*qU + w_i*(3*(c_i.(C*u))); hp = h(phi), H = theta -
 * 0.5*hp, g_0 = w_0*theta - 0.5*hp, g_i = w_i*theta + w_i*(3*(c_i.(H*u)));
 * uu = ux*ux + uy*uy, cu = c_i.u, sigma_0 = (w_0-1)*(3p) + rho0,
 * sigma_i = w_i*(3p), h_i = sigma_i + w_i*(3cu + 4.5*cu*cu - 1.5*uu).
 * Synchronous; uses a temporary device allocation. */
int dlb_equilibria(int64_t n, const double* macros, double* out, int h_quintic);

/* Device copy of n bytes (a plain streaming kernel), used to calibrate
 * bandwidth counters against a transfer of known size. */
int dlb_copy_kernel(void* dst, const void* src, size_t bytes, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Batches: many independent solvers (any grid sizes, their own physical
 * parameters; shared precision, use_ns, bc and n_sub) stepped in lockstep,
 * each kernel class as one launch over a (seed, tile) work list.
 * Every member evolves bit for bit as it would alone with the same
 * flow_fuse.  The caller owns one device buffer for the whole batch.
 * ------------------------------------------------------------------------- */
typedef struct dlb_batch* dlb_batch_handle;

/* Bytes for `count` members described by ps[0..count-1]; 0 if invalid. */
size_t dlb_batch_state_bytes(const dlb_params* ps, int count);
int dlb_batch_create(const dlb_params* ps, int count, void* dev_state, size_t bytes, void* hip_stream,
                     dlb_batch_handle* out);
int dlb_batch_destroy(dlb_batch_handle b);
/* Borrowed handle of member i (owned by the batch; never destroy it).  It
 * accepts every solver call except stepping and dlb_load: initialise with
 * dlb_init_seed / dlb_set_fields, observe with dlb_get_fields / dlb_reduce /
 * dlb_save.  NULL if i is out of range. */
dlb_handle dlb_batch_member(dlb_batch_handle b, int i);
/* Advance every member n >= 0 main steps (asynchronous; replays a captured
 * two-step HIP graph for long runs). */
int dlb_batch_step(dlb_batch_handle b, int64_t n);
int64_t dlb_batch_step_count(dlb_batch_handle b);
/* Launch configuration: flow sub-steps fused per launch (1, 3, 5) and the
 * grids as workgroups per compute unit for the node kernels and for the
 * fused flow kernel (1..4096 each; a grid with at least one workgroup per
 * tile runs one tile per workgroup, a smaller one loops its workgroups over
 * the tiles; the default is 5, 4096, 4096).  DLB_EINVAL outside these
 * ranges. */
int dlb_batch_set_config(dlb_batch_handle b, int fuse, int bpc_node, int bpc_tb);
int dlb_batch_get_config(dlb_batch_handle b, int* out3);
/* Node tile of the batched phi/C/theta and one-sub-step flow launches:
 * tile_width x (256 / tile_width) nodes, tile_width 32, 64 (default), 128 or
 * 256; every member's results are the same for each.  The fused flow
 * launch's tile is set by the fuse depth: its 64 x 32 extended tile stores a
 * (64 - 2K) x (32 - 2K) centre.  DLB_EINVAL for another width.  get returns
 * the width, or a negative error code. */
int dlb_batch_set_node_tile(dlb_batch_handle b, int tile_width);
int dlb_batch_get_node_tile(dlb_batch_handle b);
/* Autotuner: times trial_steps batch steps (HIP events) for each candidate
 * launch configuration (fuse depth and fused workgroups per CU, then node
 * workgroups per CU, then node tile shape), keeps the fastest, returns its
 * ms per step.  The trial steps consume the state: call it before
 * initialising the members (member step counters restart at 0).
 * Synchronises. */
int dlb_batch_autotune(dlb_batch_handle b, int trial_steps, double* ms_best);

const char* dlb_strerror(int code);
const char* dlb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DLB_H */
