// kernels.h -- HIP kernels for gfx950 of the diffuse-interface MRT lattice
// Boltzmann method (Zhan et al., arXiv:2209.01444).
//
// State layout in the caller's buffer (SoA, one plane per population,
// x fastest, planes padded to 64 elements):
//   pop[2][15]  phi (0-4), solute (5-9), heat (10-14) populations, ping-pong
//   flow[2][9]  flow populations (h_0 stored as h_0 - rho0), ping-pong
//   hist[6]     phi, Q, (C u)x, (C u)y, (H u)x, (H u)y of the previous step
//   options:    phin (phi^t, grad_stencil); aux[4] (u, d_t(Hu) of time t)
//               and five scratch heat planes (n_sub_t > 1)
//
// One main step (Jacobi order: every lattice reads the fields of time t):
//   k_pct      phi, C, theta collide at every node and push-stream; the
//              phi lattice uses the modified streaming of Remark 2 / Sec. 3.1;
//              the history planes are overwritten with the time-t values, so
//              hist[0] holds phi^t for the flow sub-steps that follow.
//              (k_phi_plane runs before it for the stencil-gradient option;
//              k_heat_sub x n_sub_t after it when the heat lattice takes
//              sub-steps.)
//   k_flow     x N_sub: D2Q9 MRT collision with the diffuse force of
//              Sec. 3.4 at frozen phi^t, push-streamed; or K sub-steps per
//              launch in k_flow_tbw (FP32 arithmetic) / k_flow_tb (FP64).
// Wall nodes of the channel and far-field configurations are never stored:
// whoever reads one rebuilds it from its inward neighbour (zero gradient, or
// the far-field liquid, for phi, C, H; non-equilibrium extrapolation for the
// flow).
#pragma once

#include "lattice.h"

namespace dlb {

static constexpr int C5X[5] = {0, 1, 0, -1, 0};
static constexpr int C5Y[5] = {0, 0, 1, 0, -1};
static constexpr int C9X[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static constexpr int C9Y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Destination of a push along (cx, cy): periodic wrap, or -1 when the
// destination is a wall node / outside the channel.
template <bool WALLS>
__device__ __forceinline__ long long push_dest(const KParams& kp, int x, int y, int cx, int cy) {
    int dx = x + cx, dy = y + cy;
    if constexpr (WALLS) {
        if (dx < 1 || dy < 1 || dx > kp.nx - 2 || dy > kp.ny - 2) return -1;
    } else {
        dx = dx < 0 ? dx + kp.nx : (dx >= kp.nx ? dx - kp.nx : dx);
        dy = dy < 0 ? dy + kp.ny : (dy >= kp.ny ? dy - kp.ny : dy);
    }
    return (long long)dy * kp.nx + dx;
}

// Far-field walls (Sec. 4.4; the flow lattice is off): the wall node's phi,
// C and H populations are those of its inward neighbour moved by the change
// of the equilibrium, at u = 0, from the neighbour's fields to the far-field
// liquid phi = -1, C = ff_C, theta = theta0 (non-equilibrium extrapolation).
template <class T>
__device__ __forceinline__ void farfield_rebuild(const KParams& kp, T* f, T* n, T* g) {
#pragma clang fp contract(off)
    const T phi = (((f[0] + f[1]) + f[2]) + f[3]) + f[4];
    const T C = (((n[0] + n[1]) + n[2]) + n[3]) + n[4];
    const T k = T(kp.k);
    const T U = (T(2) * C / (T(1) + k - (T(1) - k) * phi) - T(1)) / (T(1) - k);
    T eb[5], ef[5];
    eq_phi<T>(T(-1), eb);
    eq_phi<T>(phi, ef);
#pragma unroll
    for (int i = 0; i < 5; ++i) f[i] = f[i] + (eb[i] - ef[i]);
    eq_solute<T>(T(kp.ff_C), T(-1), T(kp.ff_U), T(0), T(0), eb);
    eq_solute<T>(C, phi, U, T(0), T(0), ef);
#pragma unroll
    for (int i = 0; i < 5; ++i) n[i] = n[i] + (eb[i] - ef[i]);
    if (kp.use_t) {
        const T H = (((g[0] + g[1]) + g[2]) + g[3]) + g[4];
        const T theta = H + T(0.5) * h_of(phi, kp.h_quintic);
        eq_heat<T>(T(kp.theta0), T(-1), kp.h_quintic, T(0), T(0), eb);
        eq_heat<T>(theta, phi, kp.h_quintic, T(0), T(0), ef);
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = g[i] + (eb[i] - ef[i]);
    }
}

// Non-equilibrium extrapolation (Sec. 4 preamble) of the wall node (x, y)
// from the populations hf of its inward neighbour x_f, with the frozen phi
// there: h = hf + h^eq(p_b, u_b) - h^eq(p_f, u_f), boundary values by wall;
// the equilibrium (eq_flow) difference is expanded in closed form.
template <class T, bool FORCE>
__device__ __forceinline__ FlowMacro<T> flow_macro_of(const T* h, T phi, const KParams& kp) {
    if constexpr (FORCE) return flow_macro_force(h, phi, kp);
    else return flow_macro(h, phi);
}

template <class T, bool FORCE = false>
__device__ __forceinline__ void wall_rebuild(const KParams& kp, int x, int y, const T* hf, T phi_f,
                                             T* h) {
    // no contraction: the same rounding in every kernel that inlines this
#pragma clang fp contract(off)
    FlowMacro<T> m = flow_macro_of<T, FORCE>(hf, phi_f, kp);
    T ubx, uby, pb;
    if (x == 0) {  // velocity inlet
        ubx = T(kp.uin_x_sub);
        uby = T(kp.uin_y_sub);
        pb = m.p;
    } else if (x == kp.nx - 1) {  // outflow: du/dx = 0, p = 0
        ubx = m.ux;
        uby = (y == 0 || y == kp.ny - 1) ? T(0) : m.uy;
        pb = T(0);
    } else {  // free slip
        ubx = m.ux;
        uby = T(0);
        pb = m.p;
    }
    // h^eq(p_b, u_b) - h^eq(p_f, u_f) written out with du = u_b - u_f and
    // su = u_b + u_f: w_i [A + 3 c.du + 9/2 (c.du)(c.su)] for i > 0 and
    // w_0 A - 3 dp for i = 0, where A = 3 dp - 3/2 du.su
    const T dp = pb - m.p, dx = ubx - m.ux, dy = uby - m.uy, sx = ubx + m.ux, sy = uby + m.uy;
    const T A = T(3) * dp - T(1.5) * (dx * sx + dy * sy);
    const T w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
    const T qx = T(4.5) * dx * sx, qy = T(4.5) * dy * sy;
    const T d5 = dx + dy, s5 = sx + sy, d6 = dy - dx, s6 = sy - sx;
    const T q5 = T(4.5) * d5 * s5, q6 = T(4.5) * d6 * s6;
    h[0] = hf[0] + (T(4.0 / 9.0) * A - T(3) * dp);
    h[1] = hf[1] + w1 * ((A + qx) + T(3) * dx);
    h[3] = hf[3] + w1 * ((A + qx) - T(3) * dx);
    h[2] = hf[2] + w1 * ((A + qy) + T(3) * dy);
    h[4] = hf[4] + w1 * ((A + qy) - T(3) * dy);
    h[5] = hf[5] + w2 * ((A + q5) + T(3) * d5);
    h[7] = hf[7] + w2 * ((A + q5) - T(3) * d5);
    h[6] = hf[6] + w2 * ((A + q6) + T(3) * d6);
    h[8] = hf[8] + w2 * ((A + q6) - T(3) * d6);
}

// Flow populations of node (x, y) at the current sub-step.  Interior nodes
// load them; wall nodes rebuild them from the inward neighbour x_f.
template <class T, class S, bool WALLS, bool FORCE = false>
__device__ __forceinline__ void flow_node(const KParams& kp, const S* __restrict__ h_in, int x,
                                          int y, size_t idx, T phi_f, T* h) {
    const size_t P = (size_t)kp.plane;
    if (!WALLS || !is_wall(kp, x, y)) {
#pragma unroll
        for (int i = 0; i < 9; ++i) h[i] = ld_pop<T>(h_in, i * P + idx, kp.shift[15 + i]);
        return;
    }
    size_t f = inward_idx(kp, x, y);
    T hf[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) hf[i] = ld_pop<T>(h_in, i * P + f, kp.shift[15 + i]);
    wall_rebuild<T, FORCE>(kp, x, y, hf, phi_f, h);
}

// Ablation of the local scheme: grad phi from the isotropic nine-point
// difference (1/cs^2) sum_i w_i c_i phi(x + c_i) of the node values of phi
// at time t (the plane kp.phin, written by k_phi_plane), with the bulk guard
// and anisotropy of the local scheme.  A wall node, a copy of its inward
// neighbour, takes that neighbour's gradient.
template <class T, class HT, bool WALLS>
__device__ __forceinline__ void stencil_gradient(const KParams& kp, int x, int y, T& gx, T& gy, T& a, T& Nx,
                                                 T& Ny) {
    const HT* __restrict__ ph = (const HT*)kp.phin;
    if (WALLS) {
        x = x < 1 ? 1 : (x > kp.nx - 2 ? kp.nx - 2 : x);
        y = y < 1 ? 1 : (y > kp.ny - 2 ? kp.ny - 2 : y);
    }
    // neighbours x +- 1, y +- 1 (periodic wrap; on channel grids x and y are
    // interior here, so the neighbours exist)
    const int xe = x + 1 < kp.nx ? x + 1 : 0, xw = x > 0 ? x - 1 : kp.nx - 1;
    const int yn = y + 1 < kp.ny ? y + 1 : 0, ys = y > 0 ? y - 1 : kp.ny - 1;
    const size_t r0 = (size_t)y * kp.nx, rn = (size_t)yn * kp.nx, rs = (size_t)ys * kp.nx;
    const T e = T(ph[r0 + xe]), w = T(ph[r0 + xw]), n = T(ph[rn + x]), so = T(ph[rs + x]);
    const T ne = T(ph[rn + xe]), nw = T(ph[rn + xw]), sw = T(ph[rs + xw]), se = T(ph[rs + xe]);
    // 3 w_axis = 1/3, 3 w_diagonal = 1/12
    gx = (e - w) * T(1.0 / 3.0) + ((ne - nw) + (se - sw)) * T(1.0 / 12.0);
    gy = (n - so) * T(1.0 / 3.0) + ((ne + nw) - (se + sw)) * T(1.0 / 12.0);
    if (gx * gx + gy * gy < T(GRAD_GUARD)) {
        gx = gy = T(0);
        a = T(1);
        Nx = Ny = T(0);
    } else {
        anisotropy(kp, gx, gy, a, Nx, Ny);
    }
}

// phi at time t per node into the plane phin (grad_stencil only); a wall
// node carries its inward neighbour's value (zero gradient)
template <class CF, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_phi_plane(const KParams kp, const typename CF::S* __restrict__ pin,
                                                     typename CF::H* __restrict__ phin) {
    using T = typename CF::T;
    int x, y;
    if (!node_of_thread(kp, x, y)) return;
    const size_t P = (size_t)kp.plane;
    const size_t idx = (size_t)y * kp.nx + x;
    const size_t src = (WALLS && is_wall(kp, x, y)) ? inward_idx(kp, x, y) : idx;
    T f[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) f[i] = ld_pop<T>(pin, i * P + src, kp.shift[i]);
    phin[idx] = typename CF::H((((f[0] + f[1]) + f[2]) + f[3]) + f[4]);
}

// Heat collision (Sec. 3.3) with S = diag(1, s1T, s1T, 1, 1), in closed
// form; Hu and d_t(Hu) in the time unit of the lattice's step.
template <class T>
__device__ __forceinline__ void heat_collide(T s1t, const T* g, T H, T theta, T Hux, T Huy, T dHx, T dHy, T* pg) {
    const T gf = T(1) - T(0.5) * s1t;  // (1 - s1/2) (1/3)(3 d_t(Hu))
    const T m1x = (g[1] - g[3]) - s1t * ((g[1] - g[3]) - Hux) + gf * dHx;
    const T m1y = (g[2] - g[4]) - s1t * ((g[2] - g[4]) - Huy) + gf * dHy;
    const T m3 = theta * T(1.0 / 3.0);
    pg[0] = H - T(2) * m3;
    pg[1] = T(0.5) * (m3 + m1x);
    pg[3] = T(0.5) * (m3 - m1x);
    pg[2] = T(0.5) * (m3 + m1y);
    pg[4] = T(0.5) * (m3 - m1y);
}

// One heat sub-step (multi-time-scaling for Le != 1: n_sub_t sub-steps of
// dt/n_sub_t per main step, after k_pct): phi frozen at phi^t (hist[0]),
// diffusivity alpha/n_sub_t (kp.s1t), velocity u^t/n_sub_t and the d_t(Hu)
// correction d_t(Hu)/n_sub_t^2 from the planes k_pct wrote (kp.aux);
// push-streamed like k_pct, wall nodes taking their inward neighbour's heat
// populations and their own velocity.
// gin, gout: the five heat planes of a population buffer or the scratch.
template <class CF, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_heat_sub(const KParams kp, const typename CF::SC* __restrict__ gin,
                                                    typename CF::SC* __restrict__ gout,
                                                    const typename CF::H* __restrict__ hist) {
    using T = typename CF::T;
    using HT = typename CF::H;
    int x, y;
    if (!node_of_thread(kp, x, y)) return;
    const size_t P = (size_t)kp.plane;
    const size_t idx = (size_t)y * kp.nx + x;
    const size_t src = (WALLS && is_wall(kp, x, y)) ? inward_idx(kp, x, y) : idx;
    T g[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = ld_pop<T>(gin, i * P + src, kp.shift[10 + i]);
    const T H = (((g[0] + g[1]) + g[2]) + g[3]) + g[4];
    const T phi = T(hist[idx]);
    const T theta = H + T(0.5) * h_of(phi, kp.h_quintic);
    // the node's own melt velocity (a wall node's comes from its rebuilt
    // flow populations, as in k_pct)
    const HT* __restrict__ aux = (const HT*)kp.aux;
    const T inv = T(1) / T(kp.n_sub_t);
    const T ux = T(aux[idx]) * inv, uy = T(aux[P + idx]) * inv;
    const T dHx = T(aux[2 * P + idx]) * (inv * inv), dHy = T(aux[3 * P + idx]) * (inv * inv);
    T pg[5];
    heat_collide<T>(T(kp.s1t), g, H, theta, H * ux, H * uy, dHx, dHy, pg);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        long long d = push_dest<WALLS>(kp, x, y, C5X[i], C5Y[i]);
        if (d < 0) continue;
        st_pop(gout, i * P + (size_t)d, pg[i], kp.shift[10 + i]);
    }
}

// ---------------------------------------------------------------------------
// K1: phi, C, theta main step.
// ---------------------------------------------------------------------------
template <class CF, bool NS, bool WALLS, bool FORCE = false>
__device__ __forceinline__ void pct_node(const KParams& kp, const typename CF::S* __restrict__ pin,
                                         typename CF::S* __restrict__ pout,
                                         const typename CF::S* __restrict__ hin,
                                         typename CF::H* __restrict__ hist, int hist_valid, int x,
                                         int y) {
    using T = typename CF::T;
    using HT = typename CF::H;
    using S = typename CF::S;
    const size_t P = (size_t)kp.plane;
    const size_t idx = (size_t)y * kp.nx + x;
    const bool wall = WALLS && is_wall(kp, x, y);
    const size_t src = wall ? inward_idx(kp, x, y) : idx;

    // Every load of the node is issued before its arithmetic: the kernel is
    // bound by HBM, and groups of loads each waited for in turn keep fewer
    // bytes in flight.  All fifteen population planes and the history planes
    // exist whatever the flags, so the loads are unconditional; what a flag
    // leaves unused is discarded.
    T f[5], n[5], g[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        f[i] = ld_pop<T>(pin, i * P + src, kp.shift[i]);
        n[i] = ld_pct<CF, T>(pin, 5 + i, P, src, kp.shift);
        g[i] = ld_pct<CF, T>(pin, 10 + i, P, src, kp.shift);
    }
    T hr[9];
    if constexpr (NS) {
#pragma unroll
        for (int i = 0; i < 9; ++i) hr[i] = ld_pop<T>(hin, i * P + src, kp.shift[15 + i]);
    }
    constexpr int NH = NS ? 6 : 2;
    T hv[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) hv[j] = T(hist[j * P + idx]);
    long long dst[5];
    T fold[5];
    fold[0] = f[0];
    dst[0] = push_dest<WALLS>(kp, x, y, C5X[0], C5Y[0]);
#pragma unroll
    for (int i = 1; i < 5; ++i) {
        dst[i] = push_dest<WALLS>(kp, x, y, C5X[i], C5Y[i]);
        fold[i] = ld_pop<T>(pin, i * P + (dst[i] < 0 ? idx : (size_t)dst[i]), kp.shift[i]);
    }
    if (!kp.use_t)
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = T(0);
    if constexpr (WALLS && !NS) {
        if (wall && kp.farfield) farfield_rebuild<T>(kp, f, n, g);
    }
    // macroscopic fields of time t (Sec. 3.1-3.3); isothermal runs (no heat
    // lattice) keep theta = theta0, H = theta0 - h(phi)/2
    const T phi = (((f[0] + f[1]) + f[2]) + f[3]) + f[4];
    const T C = (((n[0] + n[1]) + n[2]) + n[3]) + n[4];
    const T k = T(kp.k);
    const T hphi = h_of(phi, kp.h_quintic);
    const T H = kp.use_t ? (((g[0] + g[1]) + g[2]) + g[3]) + g[4] : T(kp.theta0) - T(0.5) * hphi;
    const T theta = kp.use_t ? H + T(0.5) * hphi : T(kp.theta0);
    const T U = (T(2) * C / (T(1) + k - (T(1) - k) * phi) - T(1)) / (T(1) - k);

    // melt velocity of time t in main-step units: N_sub (3 - phi)/4 u*
    T ux = T(0), uy = T(0);
    if constexpr (NS && FORCE) {
        T h[9];
        flow_node<T, S, WALLS, true>(kp, hin, x, y, idx, phi, h);
        const FlowMacro<T> fm = flow_macro_force(h, phi, kp);
        ux = fm.ux * T(kp.nsub_d);
        uy = fm.uy * T(kp.nsub_d);
    } else if constexpr (NS) {
        T h[9];
        if (wall) {
            wall_rebuild<T, false>(kp, x, y, hr, phi, h);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) h[i] = hr[i];
        }
        T d57 = h[5] - h[7], d68 = h[6] - h[8];
        T mx = (h[1] - h[3]) + (d57 - d68);
        T my = (h[2] - h[4]) + (d57 + d68);
        T fac = T(kp.nsub_d) * (T(3) - phi) * T(0.25);
        ux = mx * fac;
        uy = my * fac;
    }

    // local gradient, anisotropy (Sec. 2, Sec. 3.1)
    T gx, gy, a, Nx, Ny;
    if (kp.grad_stencil)
        stencil_gradient<T, HT, WALLS>(kp, x, y, gx, gy, a, Nx, Ny);
    else
        local_gradient<T>(kp, f[1] - f[3], f[2] - f[4], gx, gy, a, Nx, Ny);
    const T a2 = a * a;
    const T inv_a2 = T(1) / a2;
    const T W2t = T(kp.W2t);
    const T s1 = T(1) / (T(3) * a2 * W2t + T(0.5));

    // coupling source and time derivatives (backward differences)
    const T om = T(1) - phi * phi;
    const T Q = phi * om - T(kp.lambda) * (theta + T(kp.Mcinf) * U) * om * om;
    T dQ = T(0), dphi = T(0), dCx = T(0), dCy = T(0), dHx = T(0), dHy = T(0);
    const T Cux = C * ux, Cuy = C * uy, Hux = H * ux, Huy = H * uy;
    if (hist_valid) {
        dphi = phi - hv[0];
        dQ = Q - hv[1];
        if constexpr (NS) {
            dCx = Cux - hv[2];
            dCy = Cuy - hv[3];
            dHx = Hux - hv[4];
            dHy = Huy - hv[5];
        }
    }
    hist[idx] = HT(phi);
    hist[P + idx] = HT(Q);
    if constexpr (NS) {
        hist[2 * P + idx] = HT(Cux);
        hist[3 * P + idx] = HT(Cuy);
        hist[4 * P + idx] = HT(Hux);
        hist[5 * P + idx] = HT(Huy);
    }

    // ---- phi lattice (Sec. 3.1): S = diag(1, s1, s1, 1, 1) ----
    T pf[5];
    {
        const T A = (Q + T(0.5) * a2 * dQ) * T(kp.inv_tau0);  // F + (a^2/2) d_t F, summed
        const T gfac = (T(1) - T(0.5) * s1) * T(-1.0 / 3.0) * inv_a2;  // (1 - s1/2) sum c G
        const T m1x = (T(1) - s1) * (f[1] - f[3]) + gfac * Nx;
        const T m1y = (T(1) - s1) * (f[2] - f[4]) + gfac * Ny;
        const T m3 = (phi + A) * T(1.0 / 3.0);
        pf[0] = m3;  // m0 - m3 - m4 with m0 = phi + A
        pf[1] = T(0.5) * (m3 + m1x);
        pf[3] = T(0.5) * (m3 - m1x);
        pf[2] = T(0.5) * (m3 + m1y);
        pf[4] = T(0.5) * (m3 - m1y);
    }

    // anti-trapping current (Sec. 2)
    T Jx = T(0), Jy = T(0);
    {
        T gn2 = gx * gx + gy * gy;
        if (gn2 > T(0)) {
            T c = -T(kp.jat) * (T(1) + (T(1) - k) * U) * dphi / sqrt(gn2);
            Jx = c * gx;
            Jy = c * gy;
        }
    }

    // ---- solute lattice (Sec. 3.2): S = diag(1, s1C, s1C, 1, 1) ----
    T pn[5];
    {
        const T s1c = T(kp.s1c);
        const T qU = T(0.5) * (T(1) - phi) * U;
        const T invD = T(kp.invD);
        const T Vx = T(3) * dCx - T(0.5) * U * gx + Jx * invD;
        const T Vy = T(3) * dCy - T(0.5) * U * gy + Jy * invD;
        const T gf = (T(1) - T(0.5) * s1c) * T(1.0 / 3.0);
        const T m1x = (n[1] - n[3]) - s1c * ((n[1] - n[3]) - Cux) + gf * Vx;
        const T m1y = (n[2] - n[4]) - s1c * ((n[2] - n[4]) - Cuy) + gf * Vy;
        const T m3 = qU * T(1.0 / 3.0);
        pn[0] = C - T(2) * m3;
        pn[1] = T(0.5) * (m3 + m1x);
        pn[3] = T(0.5) * (m3 - m1x);
        pn[2] = T(0.5) * (m3 + m1y);
        pn[4] = T(0.5) * (m3 - m1y);
    }

    // ---- heat lattice (Sec. 3.3), here unless it takes sub-steps ----
    T pg[5];
    heat_collide<T>(T(kp.s1t), g, H, theta, Hux, Huy, dHx, dHy, pg);
    const bool heat_here = kp.use_t && kp.n_sub_t == 1;
    if (kp.use_t && kp.n_sub_t > 1) {
        // inputs of the heat sub-steps (k_heat_sub): u and d_t(Hu) of time t
        HT* __restrict__ aux = (HT*)kp.aux;
        aux[idx] = HT(ux);
        aux[P + idx] = HT(uy);
        aux[2 * P + idx] = HT(dHx);
        aux[3 * P + idx] = HT(dHy);
    }

    // ---- streaming (push).  phi: f(y,t+1) = f(y,t) + (post - f(y,t)) / a_s^2 ----
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const long long d = dst[i];
        if (d < 0) continue;
        st_pop(pout, i * P + (size_t)d, fold[i] + (pf[i] - fold[i]) * inv_a2, kp.shift[i]);
        st_pct<CF>(pout, 5 + i, P, (size_t)d, pn[i], kp.shift);
        if (heat_here) st_pct<CF>(pout, 10 + i, P, (size_t)d, pg[i], kp.shift);
    }
}

template <class CF, bool NS, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_pct(const KParams kp, const typename CF::S* __restrict__ pin,
                                               typename CF::S* __restrict__ pout,
                                               const typename CF::S* __restrict__ hin,
                                               typename CF::H* __restrict__ hist, int hist_valid) {
    int x, y;
    if (!node_of_thread(kp, x, y)) return;
    pct_node<CF, NS, WALLS>(kp, pin, pout, hin, hist, hist_valid, x, y);
}

// The same with the external force of Sec. 3.4 in the melt velocity.
template <class CF, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_pct_force(const KParams kp, const typename CF::S* __restrict__ pin,
                                                     typename CF::S* __restrict__ pout,
                                                     const typename CF::S* __restrict__ hin,
                                                     typename CF::H* __restrict__ hist, int hist_valid) {
    int x, y;
    if (!node_of_thread(kp, x, y)) return;
    pct_node<CF, true, WALLS, true>(kp, pin, pout, hin, hist, hist_valid, x, y);
}

// ---------------------------------------------------------------------------
// K2: one flow sub-step (Sec. 3.4) at frozen phi^t (= hist[0]).
// ---------------------------------------------------------------------------
template <class CF, bool WALLS, bool FORCE = false>
__device__ __forceinline__ void flow_step_node(const KParams& kp, const typename CF::S* __restrict__ hin,
                                               typename CF::S* __restrict__ hout,
                                               const typename CF::H* __restrict__ phi_t, int x, int y) {
    using T = typename CF::T;
    using S = typename CF::S;
    const size_t P = (size_t)kp.plane;
    const size_t idx = (size_t)y * kp.nx + x;
    const T phi = T(phi_t[idx]);
    T h[9];
    T phi_f = phi;
    if (WALLS && is_wall(kp, x, y)) phi_f = T(phi_t[inward_idx(kp, x, y)]);
    flow_node<T, S, WALLS, FORCE>(kp, hin, x, y, idx, phi_f, h);
    T o[9];
    if constexpr (FORCE) flow_collide_force<T>(h, phi, kp, T(kp.s2u), o);
    else flow_collide<T>(h, flow_coef(phi), T(kp.s2u), o);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        long long d = push_dest<WALLS>(kp, x, y, C9X[i], C9Y[i]);
        if (d < 0) continue;
        st_pop(hout, i * P + (size_t)d, o[i], kp.shift[15 + i]);
    }
}

template <class CF, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_flow(const KParams kp, const typename CF::S* __restrict__ hin,
                                                typename CF::S* __restrict__ hout,
                                                const typename CF::H* __restrict__ phi_t) {
    int x, y;
    if (!node_of_thread(kp, x, y)) return;
    flow_step_node<CF, WALLS>(kp, hin, hout, phi_t, x, y);
}

// One flow sub-step with the external force and varphi of Sec. 3.4.
template <class CF, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_flow_force(const KParams kp, const typename CF::S* __restrict__ hin,
                                                      typename CF::S* __restrict__ hout,
                                                      const typename CF::H* __restrict__ phi_t) {
    int x, y;
    if (!node_of_thread(kp, x, y)) return;
    flow_step_node<CF, WALLS, true>(kp, hin, hout, phi_t, x, y);
}

// ---------------------------------------------------------------------------
// K2': K fused flow sub-steps per launch (temporal blocking).  A workgroup
// holds an extended tile of EX x EY nodes, one per thread, with the
// populations in registers.  Each sub-step: collide, write the post-collision
// populations to LDS, pull the streamed ones back from the neighbours' LDS
// slots (wall nodes instead rebuild theirs from the inward neighbour's pulled
// populations, read from the same LDS slots).  Values near the tile edge go
// stale by one ring per sub-step, so after K sub-steps the central
// (EX-2K) x (EY-2K) nodes are exact and are stored, aligned, to the output
// buffer.  Arithmetic per node and sub-step is that of k_flow.
// ---------------------------------------------------------------------------
template <int EX, int EY, int K> struct TbShape {
    static constexpr int OX = EX - 2 * K, OY = EY - 2 * K;
};
// extended tile per arithmetic type: 9 LDS planes of EX*EY values stay at
// 36 KiB (32x32 in FP32, 32x16 in FP64)
template <class T> struct TbTile;
template <> struct TbTile<float> { static constexpr int EX = 32, EY = 32; };
template <> struct TbTile<double> { static constexpr int EX = 32, EY = 16; };

template <class CF, bool WALLS, int EX, int EY, int K>
__device__ __forceinline__ void flow_tb_tile(const KParams& kp, const typename CF::S* __restrict__ hin,
                                             typename CF::S* __restrict__ hout,
                                             const typename CF::H* __restrict__ phi_t, int bx, int by) {
    using T = typename CF::T;
    using S = typename CF::S;
    constexpr int OX = TbShape<EX, EY, K>::OX, OY = TbShape<EX, EY, K>::OY;
    __shared__ T lds[9][EY][EX];
    const size_t P = (size_t)kp.plane;
    const int tx = threadIdx.x % EX, ty = threadIdx.x / EX;
    int gx = bx * OX - K + tx, gy = by * OY - K + ty;
    bool exists = true;
    if constexpr (WALLS) {
        exists = gx >= 0 && gy >= 0 && gx < kp.nx && gy < kp.ny;
    } else {
        gx = gx < 0 ? gx + kp.nx : (gx >= kp.nx ? gx - kp.nx : gx);
        gy = gy < 0 ? gy + kp.ny : (gy >= kp.ny ? gy - kp.ny : gy);
    }
    const bool wall = WALLS && exists && is_wall(kp, gx, gy);
    const size_t idx = exists ? (size_t)gy * kp.nx + gx : 0;
    // local coordinates of the inward neighbour (wall nodes only)
    int fx = tx, fy = ty;
    T phi = T(0), phi_f = T(0);
    T h[9];
    if (exists) {
        phi = T(phi_t[idx]);
        phi_f = phi;
        if (wall) {
            int xf = gx < 1 ? 1 : (gx > kp.nx - 2 ? kp.nx - 2 : gx);
            int yf = gy < 1 ? 1 : (gy > kp.ny - 2 ? kp.ny - 2 : gy);
            fx = tx + (xf - gx);
            fy = ty + (yf - gy);
            phi_f = T(phi_t[(size_t)yf * kp.nx + xf]);
        }
        flow_node<T, S, WALLS>(kp, hin, gx, gy, idx, phi_f, h);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) h[i] = T(0);
    }
    const T s2 = T(kp.s2u);
    const FlowCoef<T> fc = flow_coef(phi);
    for (int sub = 0; sub < K; ++sub) {
        T o[9];
        flow_collide<T>(h, fc, s2, o);
#pragma unroll
        for (int i = 0; i < 9; ++i) lds[i][ty][tx] = o[i];
        __syncthreads();
        // pull: source (x - c_i) of this node, or of the inward neighbour
        const int px = wall ? fx : tx, py = wall ? fy : ty;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int sx = px - C9X[i], sy = py - C9Y[i];
            sx = sx < 0 ? 0 : (sx > EX - 1 ? EX - 1 : sx);  // stale ring: any in-tile slot
            sy = sy < 0 ? 0 : (sy > EY - 1 ? EY - 1 : sy);
            h[i] = lds[i][sy][sx];
        }
        if (WALLS && wall) {
            // rebuild from the inward neighbour's pulled populations
            T hf[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) hf[i] = h[i];
            wall_rebuild(kp, gx, gy, hf, phi_f, h);
        }
        __syncthreads();
    }
    const bool out = tx >= K && tx < EX - K && ty >= K && ty < EY - K;
    const int ox = bx * OX + (tx - K), oy = by * OY + (ty - K);
    if (out && exists && !wall && ox < kp.nx && oy < kp.ny) {
#pragma unroll
        for (int i = 0; i < 9; ++i) st_pop(hout, i * P + idx, h[i], kp.shift[15 + i]);
    }
}

// ---------------------------------------------------------------------------
// K2'' (FP32 arithmetic): the same K fused sub-steps with a wave-row tile.
// The extended tile is 64 x (NW R) nodes: wave w owns rows [w R, w R + R),
// lane l column l, each thread R nodes of one column in registers.  After a
// collision, streaming along x is a one-lane shift of the wave (DPP), along y
// a move between the thread's own rows; only the first and last row of each
// wave cross to the neighbouring waves, through a small double-buffered LDS
// exchange (one barrier per sub-step).  Arithmetic per node and sub-step is
// that of k_flow.
//
// Walls (channel, edge tiles only) need no further barrier.  The tiling is
// shifted by kp.tbw_dy rows so that a wall row y = 0 or ny - 1 always lies in
// the same wave as its inward row: its nodes take that row's pulled
// populations from the thread's own registers.  The wall columns x = 0 and
// nx - 1 are then rebuilt by one pass per wave: the lane of the inward column
// writes its R rows to a per-wave LDS slot, lanes 0-7 rebuild one (side,
// row) pair each (a corner from the row inward of it: the diagonal
// neighbour), and the wall lane reads the results back.  Tiles whose
// extended region holds no wall node run the variant without walls
// (flow_tbw_tile_any).
// ---------------------------------------------------------------------------
template <int NW_> struct TbWaveT {
    static constexpr int NW = NW_, R = 4, EX = 64, EY = NW_ * R;
};
// the tile of 8 waves (64 x 32 nodes), and the tall one of 12 (64 x 48): less
// halo per stored node, fewer tiles resident per compute unit; the host takes
// the tall one where a grid has enough tiles to fill several rounds
using TbWave = TbWaveT<8>;
constexpr int TBW_TALL_NW = 12;

// Row shift of the wave-row tiling for K fused sub-steps (tile origin
// y = by OY - K - dy): the smallest tile count among shifts dy in [0, 2R)
// for which every wall row falling into a tile has its inward row in the
// same wave.  Returns dy (0 without walls) and sets *nby; -1 if none.
inline int tbw_row_shift(int ny, int K, bool walls, int* nby, int EY = TbWave::EY) {
    constexpr int R = TbWave::R;
    const int OY = EY - 2 * K;
    if (!walls) {
        *nby = (ny + OY - 1) / OY;
        return 0;
    }
    int best = -1, best_n = 0;
    for (int dy = 0; dy < 2 * R; ++dy) {
        const int n = (ny + dy + OY - 1) / OY;
        bool ok = true;
        for (int by = 0; by < n && ok; ++by) {
            const int y0 = by * OY - K - dy;
            const int t = -y0, b = ny - 1 - y0;
            if (t >= 0 && t < EY) ok = t + 1 < EY && (t + 1) / R == t / R;
            if (ok && b >= 0 && b < EY) ok = b >= 1 && (b - 1) / R == b / R;
        }
        if (ok && (best < 0 || n < best_n)) {
            best = dy;
            best_n = n;
        }
    }
    *nby = best_n;
    return best;
}

// DPP wave shifts: lane l receives the value of lane l - 1 (from_left) or
// l + 1 (from_right); the edge lane receives 0 (a stale column).
__device__ __forceinline__ float lane_from_left(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_right(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// orders this wave's LDS writes before its later LDS reads (lanes exchange
// data through LDS within one wave)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of a wave-row tile, one block per workgroup whichever tile variant
// runs: exchange slots [buffer][wave][k][lane] (k 0-2 the up-movers 2, 5, 6
// of the wave's last row, k 3-5 the down-movers 4, 7, 8 of its first row)
// and the wall-column pass [wave][side (west, east)][row][population],
// rows padded to 12 floats
template <int NW> struct TbwLds {
    float xch[2][NW][6][64];
    float xw_in[NW][2][TbWave::R][12];
    float xw_out[NW][2][TbWave::R][12];
};
template <int NW> __device__ __forceinline__ TbwLds<NW>& tbw_lds() {
    __shared__ TbwLds<NW> l;
    return l;
}

template <class CF, bool WALLS, int K, int NW_ = TbWave::NW>
__device__ __forceinline__ void flow_tbw_tile(const KParams& kp, const typename CF::S* __restrict__ hin,
                                              typename CF::S* __restrict__ hout,
                                              const typename CF::H* __restrict__ phi_t, int bx, int by) {
    using T = typename CF::T;
    using S = typename CF::S;
    using TW = TbWaveT<NW_>;
    static_assert(sizeof(T) == 4, "wave-row tile is for FP32 arithmetic");
    constexpr int NW = TW::NW, R = TW::R, EX = TW::EX, EY = TW::EY;
    constexpr int OX = EX - 2 * K, OY = EY - 2 * K;
    TbwLds<NW>& lds = tbw_lds<NW>();
    auto& xch = lds.xch;
    auto& xw_in = lds.xw_in;
    auto& xw_out = lds.xw_out;
    const size_t P = (size_t)kp.plane;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int X0 = bx * OX - K, Y0 = by * OY - K - kp.tbw_dy[NW != TbWave::NW][K == 5];  // 0 without walls
    int gx = X0 + lane;
    bool xin = true;
    if constexpr (WALLS) {
        xin = gx >= 0 && gx < kp.nx;
    } else {
        gx = gx < 0 ? gx + kp.nx : (gx >= kp.nx ? gx - kp.nx : gx);
    }
    // tile-uniform wall geometry (channel only): wall lanes of x = 0 and
    // x = nx - 1, local rows of y = 0 and y = ny - 1
    const bool west_tile = WALLS && X0 <= 0, east_tile = WALLS && X0 + EX - 1 >= kp.nx - 1;
    const bool xwall_tile = west_tile || east_tile;
    const int lane_w = -X0, lane_e = kp.nx - 1 - X0;
    const int top_row = -Y0, bot_row = kp.ny - 1 - Y0;
    const bool top_tile = WALLS && top_row >= 0 && top_row < EY;
    const bool bot_tile = WALLS && bot_row >= 0 && bot_row < EY;
    T h[R][9];
    T phi_yw = T(0);  // frozen phi inward of this wave's wall row y = 0 or ny - 1
    FlowCoef<T> fc[R];
    bool liq[R];
    int gy[R];
    bool ex[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int y = Y0 + w * R + r;
        bool e = xin;
        if constexpr (WALLS) {
            e = e && y >= 0 && y < kp.ny;
        } else {
            y = y < 0 ? y + kp.ny : (y >= kp.ny ? y - kp.ny : y);
        }
        gy[r] = y;
        ex[r] = e;
        T phi = T(0);
        if (e) {
            const size_t idx = (size_t)y * kp.nx + gx;
            phi = T(phi_t[idx]);
            T phi_f = phi;
            if (WALLS && is_wall(kp, gx, y)) phi_f = T(phi_t[inward_idx(kp, gx, y)]);
            if (WALLS && (y == 0 || y == kp.ny - 1)) phi_yw = phi_f;
            flow_node<T, S, WALLS>(kp, hin, gx, y, idx, phi_f, h[r]);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) h[r][i] = T(0);
        }
        fc[r] = flow_coef(phi);
        liq[r] = __ballot(phi == T(-1)) == __ballot(1);  // wave-uniform: every lane of the row in the melt
    }
    // rebuild lanes of the wall-column pass: lane j < 8 takes side j / R,
    // row j % R of this wave; the frozen phi of that node's inward neighbour
    // waits in the padding of its output slot
    if constexpr (WALLS) {
        const int xw_side = lane / R, xw_row = lane % R, xw_y = Y0 + w * R + xw_row;
        if (xwall_tile && lane < 2 * R && (xw_side ? east_tile : west_tile) && xw_y >= 0 && xw_y < kp.ny)
            xw_out[w][xw_side][xw_row][9] = T(phi_t[inward_idx(kp, xw_side ? kp.nx - 1 : 0, xw_y)]);
    }
    const T s2 = T(kp.s2u);
#pragma unroll
    for (int sub = 0; sub < K; ++sub) {
        const int buf = sub & 1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            T o[9];
            if (liq[r])
                flow_collide<T, true>(h[r], fc[r], s2, o);
            else
                flow_collide<T>(h[r], fc[r], s2, o);
            // x streaming: c_x = +1 from the left lane, c_x = -1 from the right lane
            h[r][0] = o[0];
            h[r][2] = o[2];
            h[r][4] = o[4];
            h[r][1] = lane_from_left(o[1]);
            h[r][5] = lane_from_left(o[5]);
            h[r][8] = lane_from_left(o[8]);
            h[r][3] = lane_from_right(o[3]);
            h[r][6] = lane_from_right(o[6]);
            h[r][7] = lane_from_right(o[7]);
        }
        xch[buf][w][0][lane] = h[R - 1][2];
        xch[buf][w][1][lane] = h[R - 1][5];
        xch[buf][w][2][lane] = h[R - 1][6];
        xch[buf][w][3][lane] = h[0][4];
        xch[buf][w][4][lane] = h[0][7];
        xch[buf][w][5][lane] = h[0][8];
        __syncthreads();
        // y streaming: c_y = +1 from the row below (index r - 1), c_y = -1
        // from the row above (r + 1); the tile's outer rows keep stale values
        {
            const int wd = w > 0 ? w - 1 : 0, wu = w < NW - 1 ? w + 1 : NW - 1;
            T up2 = xch[buf][wd][0][lane], up5 = xch[buf][wd][1][lane], up6 = xch[buf][wd][2][lane];
            T dn4 = xch[buf][wu][3][lane], dn7 = xch[buf][wu][4][lane], dn8 = xch[buf][wu][5][lane];
#pragma unroll
            for (int r = R - 1; r > 0; --r) {
                h[r][2] = h[r - 1][2];
                h[r][5] = h[r - 1][5];
                h[r][6] = h[r - 1][6];
            }
            h[0][2] = up2;
            h[0][5] = up5;
            h[0][6] = up6;
#pragma unroll
            for (int r = 0; r < R - 1; ++r) {
                h[r][4] = h[r + 1][4];
                h[r][7] = h[r + 1][7];
                h[r][8] = h[r + 1][8];
            }
            h[R - 1][4] = dn4;
            h[R - 1][7] = dn7;
            h[R - 1][8] = dn8;
        }
        if constexpr (WALLS) {
            // y walls: the inward row is in this wave (row shift of the tiling)
            if (top_tile || bot_tile) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int lr = w * R + r;
                    const bool yt = top_tile && lr == top_row, yb = bot_tile && lr == bot_row;
                    if (!(yt || yb)) continue;  // wave-uniform
                    T hf[9];
#pragma unroll
                    for (int i = 0; i < 9; ++i) hf[i] = yt ? h[r + 1 < R ? r + 1 : r][i] : h[r >= 1 ? r - 1 : r][i];
                    if (ex[r]) wall_rebuild(kp, gx, gy[r], hf, phi_yw, h[r]);
                }
            }
            // x walls: one rebuild pass per wave through LDS
            if (xwall_tile) {
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    if (!(side ? east_tile : west_tile)) continue;  // tile-uniform
                    const int lane_in = side ? lane_e - 1 : lane_w + 1;
                    if (lane == lane_in) {
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int i = 0; i < 9; ++i) xw_in[w][side][r][i] = h[r][i];
                    }
                }
                wave_lds_sync();
                const int xw_side = lane / R, xw_row = lane % R, xw_y = Y0 + w * R + xw_row;
                if (lane < 2 * R && (xw_side ? east_tile : west_tile) && xw_y >= 0 && xw_y < kp.ny) {
                    // a corner takes the row inward of it (same wave by the row shift)
                    const int lr = w * R + xw_row;
                    const int src = (top_tile && lr == top_row) ? xw_row + 1
                                                                : ((bot_tile && lr == bot_row) ? xw_row - 1 : xw_row);
                    T hf[9], hw[9];
#pragma unroll
                    for (int i = 0; i < 9; ++i) hf[i] = xw_in[w][xw_side][src][i];
                    wall_rebuild(kp, xw_side ? kp.nx - 1 : 0, xw_y, hf, T(xw_out[w][xw_side][xw_row][9]), hw);
#pragma unroll
                    for (int i = 0; i < 9; ++i) xw_out[w][xw_side][xw_row][i] = hw[i];
                }
                wave_lds_sync();
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    if (!(side ? east_tile : west_tile)) continue;
                    if (lane == (side ? lane_e : lane_w)) {
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            if (!ex[r]) continue;
#pragma unroll
                            for (int i = 0; i < 9; ++i) h[r][i] = xw_out[w][side][r][i];
                        }
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int lr = w * R + r;
        const bool out = lane >= K && lane < EX - K && lr >= K && lr < EY - K;
        const int ox = bx * OX + (lane - K), oy = Y0 + lr;
        if (out && ex[r] && !(WALLS && is_wall(kp, gx, gy[r])) && ox < kp.nx && oy < kp.ny) {
            const size_t idx = (size_t)gy[r] * kp.nx + gx;
#pragma unroll
            for (int i = 0; i < 9; ++i) st_pop(hout, i * P + idx, h[r][i], kp.shift[15 + i]);
        }
    }
}

// A wave-row tile of a channel grid whose extended region holds no wall
// node runs the tile code without walls (no bounds or wall tests, fewer
// registers live): same arithmetic, same results.
template <class CF, bool WALLS, int K, int NW = TbWave::NW>
__device__ __forceinline__ void flow_tbw_tile_any(const KParams& kp, const typename CF::S* __restrict__ hin,
                                                  typename CF::S* __restrict__ hout,
                                                  const typename CF::H* __restrict__ phi_t, int bx, int by) {
    if constexpr (WALLS) {
        using TW = TbWaveT<NW>;
        constexpr int EX = TW::EX, EY = TW::EY, OX = EX - 2 * K, OY = EY - 2 * K;
        const int X0 = bx * OX - K, Y0 = by * OY - K - kp.tbw_dy[NW != TbWave::NW][K == 5];
        if (X0 >= 1 && X0 + EX - 1 <= kp.nx - 2 && Y0 >= 1 && Y0 + EY - 1 <= kp.ny - 2) {
            flow_tbw_tile<CF, false, K, NW>(kp, hin, hout, phi_t, bx, by);
            return;
        }
    }
    flow_tbw_tile<CF, WALLS, K, NW>(kp, hin, hout, phi_t, bx, by);
}

// Tile geometry of the fused flow launch per arithmetic type: the wave-row
// tile for FP32, the LDS tile for FP64.
template <class T> struct TbGeom;
template <> struct TbGeom<float> {
    static constexpr int EX = TbWave::EX, EY = TbWave::EY, THREADS = 64 * TbWave::NW;
};
template <> struct TbGeom<double> {
    static constexpr int EX = TbTile<double>::EX, EY = TbTile<double>::EY, THREADS = EX * EY;
};

// one fused tile of either kind
template <class CF, bool WALLS, int K>
__device__ __forceinline__ void flow_fused_tile(const KParams& kp, const typename CF::S* __restrict__ hin,
                                                typename CF::S* __restrict__ hout,
                                                const typename CF::H* __restrict__ phi_t, int bx, int by) {
    using T = typename CF::T;
    if constexpr (sizeof(T) == 4)
        flow_tbw_tile_any<CF, WALLS, K>(kp, hin, hout, phi_t, bx, by);
    else
        flow_tb_tile<CF, WALLS, TbTile<T>::EX, TbTile<T>::EY, K>(kp, hin, hout, phi_t, bx, by);
}

// Tile of workgroup b.  Periodic grids: XCD-contiguous order.  Channel
// grids: the tiles on the domain edge (whose wall handling costs more) come
// first, so they start early and do not trail the launch, then the interior
// tiles in XCD-contiguous order (the first group is padded to a multiple of
// the 8 XCDs so that block b keeps running on XCD b mod 8).
template <bool WALLS>
__device__ __forceinline__ void tbw_tile_of(int b, int nbx, int nby, int& bx, int& by) {
    const int nb = nbx * nby;
    if (!WALLS || nbx <= 2 || nby <= 2) {
        const int t = xcd_remap(b, nb);
        bx = t % nbx;
        by = t / nbx;
        return;
    }
    const int E = 2 * nbx + 2 * (nby - 2), E8 = (E + 7) & ~7;
    const int o = b < E8 ? b : E8 + xcd_remap(b - E8, nb - E8);
    if (o < nbx) {
        bx = o, by = 0;
    } else if (o < 2 * nbx) {
        bx = o - nbx, by = nby - 1;
    } else if (o < E - (nby - 2)) {
        bx = 0, by = 1 + o - 2 * nbx;
    } else if (o < E) {
        bx = nbx - 1, by = 1 + o - (E - (nby - 2));
    } else {
        const int u = o - E;
        bx = 1 + u % (nbx - 2);
        by = 1 + u / (nbx - 2);
    }
}

template <class CF, bool WALLS, int K, int NW = TbWave::NW>
__global__ __launch_bounds__(64 * NW) void k_flow_tbw(const KParams kp, const typename CF::S* __restrict__ hin,
                                                      typename CF::S* __restrict__ hout,
                                                      const typename CF::H* __restrict__ phi_t, int nbx,
                                                      int nblocks) {
    int bx, by;
    tbw_tile_of<WALLS>(blockIdx.x, nbx, nblocks / nbx, bx, by);
    flow_tbw_tile_any<CF, WALLS, K, NW>(kp, hin, hout, phi_t, bx, by);
}

template <class CF, bool WALLS, int EX, int EY, int K>
__global__ __launch_bounds__(EX* EY) void k_flow_tb(const KParams kp,
                                                    const typename CF::S* __restrict__ hin,
                                                    typename CF::S* __restrict__ hout,
                                                    const typename CF::H* __restrict__ phi_t, int nbx,
                                                    int nblocks) {
    const int t = xcd_remap(blockIdx.x, nblocks);
    flow_tb_tile<CF, WALLS, EX, EY, K>(kp, hin, hout, phi_t, t % nbx, t / nbx);
}

// ---------------------------------------------------------------------------
// Initialisation (Sec. 4 preamble) and re-initialisation at given fields.
// ---------------------------------------------------------------------------
__global__ void k_seed_phi(const KParams kp, const double* __restrict__ noise,
                           double* __restrict__ phi) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t N = (size_t)kp.nx * kp.ny;
    if (i >= N) return;
    int x = (int)(i % kp.nx), y = (int)(i / kp.nx);
    double dx = x - kp.seed_x, dy = y - kp.seed_y;
    double d = sqrt(dx * dx + dy * dy);
    double v = tanh((kp.seed_R - d) / (sqrt(2.0) * kp.W0));
    if (noise && fabs(v) < 0.9) v += kp.noise_amp * noise[i];
    phi[i] = v;
}

struct InitFields {
    const double *phi, *C, *theta, *ux, *uy;  // device, nullable except phi
    double C0, U0, theta0, uin_x, uin_y;
    int c_init_U, use_ns;
    unsigned flags;          // DLB_KEEP_FLOW (1) | DLB_KEEP_NONEQ (2)
    int hist_valid;          // KEEP_NONEQ: hist holds rates (see k_restart_prep)
    const double* phi_old;   // KEEP_NONEQ: phi of the current state (k_restart_prep)
    int phi_static;          // frozen solid: the flow sub-steps read phi from hist[0]
};

constexpr unsigned KEEP_FLOW = 1u, KEEP_NONEQ = 2u;

// Isotropic D2Q9 central difference of a node field F: grad = 3 sum_i w_i c_i
// F(x + c_i), wrapped (periodic) or clamped at the channel walls.
template <bool WALLS>
__device__ __forceinline__ void cd_gradient(const KParams& kp, const double* __restrict__ F, int x,
                                            int y, double& gx, double& gy) {
    gx = 0.0;
    gy = 0.0;
    for (int i = 1; i < 9; ++i) {
        int xx = x + C9X[i], yy = y + C9Y[i];
        if (WALLS) {
            xx = xx < 0 ? 0 : (xx > kp.nx - 1 ? kp.nx - 1 : xx);
            yy = yy < 0 ? 0 : (yy > kp.ny - 1 ? kp.ny - 1 : yy);
        } else {
            xx = xx < 0 ? xx + kp.nx : (xx >= kp.nx ? xx - kp.nx : xx);
            yy = yy < 0 ? yy + kp.ny : (yy >= kp.ny ? yy - kp.ny : yy);
        }
        double w = i < 5 ? 1.0 / 9.0 : 1.0 / 36.0;
        double v = F[(size_t)yy * kp.nx + xx];
        gx += 3.0 * w * C9X[i] * v;
        gy += 3.0 * w * C9Y[i] * v;
    }
}

// First moment of the phi populations that the local gradient scheme
// (Sec. 3.1) maps back to the gradient (gx, gy).
__device__ __forceinline__ void phi_first_moment(const KParams& kp, double gx, double gy, double& Vx,
                                                 double& Vy) {
    Vx = 0.0;
    Vy = 0.0;
    if (gx * gx + gy * gy >= GRAD_GUARD) {
        double a, Nx, Ny;
        anisotropy<double>(kp, gx, gy, a, Nx, Ny);
        double s1 = 1.0 / (3.0 * a * a * kp.W2t + 0.5);
        Vx = -gx / (3.0 * s1) - kp.W2t * Nx;
        Vy = -gy / (3.0 * s1) - kp.W2t * Ny;
    }
}

// Melt velocity in main-step units from the flow populations h at phi, as a
// main step evaluates it: N_sub (3 - phi)/4 u*.
__device__ __forceinline__ void step_velocity(const KParams& kp, const double* h, double phi,
                                              double& ux, double& uy) {
    double d57 = h[5] - h[7], d68 = h[6] - h[8];
    double mx = (h[1] - h[3]) + (d57 - d68);
    double my = (h[2] - h[4]) + (d57 + d68);
    if (kp.force) {  // u* = sum c h + F/2
        mx += 0.5 * kp.fx_sub;
        my += 0.5 * kp.fy_sub;
    }
    double fac = kp.nsub_d * (3.0 - phi) * 0.25;
    ux = mx * fac;
    uy = my * fac;
}

// Restart with KEEP_NONEQ, pass 1 (reads the state, writes no population):
// phi of every node (walls rebuilt from the inward node) into phi_old, and,
// with a valid history, the time-derivative numerators value - history of
// phi, Q, Cu, Hu into the history planes at interior nodes.
template <class CF, bool NS, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_restart_prep(const KParams kp,
                                                        const typename CF::S* __restrict__ pop,
                                                        const typename CF::S* __restrict__ flow,
                                                        typename CF::H* __restrict__ hist,
                                                        double* __restrict__ phi_old, int hist_valid) {
    using HT = typename CF::H;
    int x, y;
    if (!node_of_thread(kp, x, y)) return;
    const size_t P = (size_t)kp.plane;
    const size_t idx = (size_t)y * kp.nx + x;
    const bool wall = WALLS && is_wall(kp, x, y);
    const size_t src = wall ? inward_idx(kp, x, y) : idx;
    double phi = 0.0, C = 0.0, H = 0.0;
    for (int i = 0; i < 5; ++i) {
        phi += ld_pop<double>(pop, i * P + src, kp.shift[i]);
        C += ld_pct<CF, double>(pop, 5 + i, P, src, kp.shift);
        H += ld_pct<CF, double>(pop, 10 + i, P, src, kp.shift);
    }
    phi_old[idx] = (wall && kp.farfield) ? -1.0 : phi;
    if (!hist_valid || wall) return;
    const double k = kp.k;
    const double U = (2.0 * C / (1.0 + k - (1.0 - k) * phi) - 1.0) / (1.0 - k);
    const double theta = H + 0.5 * h_of(phi, kp.h_quintic);
    const double om = 1.0 - phi * phi;
    const double Q = phi * om - kp.lambda * (theta + kp.Mcinf * U) * om * om;
    hist[idx] = HT(phi - (double)hist[idx]);
    hist[P + idx] = HT(Q - (double)hist[P + idx]);
    if constexpr (NS) {
        double h[9], ux, uy;
        for (int i = 0; i < 9; ++i) h[i] = ld_pop<double>(flow, i * P + idx, kp.shift[15 + i]);
        step_velocity(kp, h, phi, ux, uy);
        hist[2 * P + idx] = HT(C * ux - (double)hist[2 * P + idx]);
        hist[3 * P + idx] = HT(C * uy - (double)hist[3 * P + idx]);
        hist[4 * P + idx] = HT(H * ux - (double)hist[4 * P + idx]);
        hist[5 * P + idx] = HT(H * uy - (double)hist[5 * P + idx]);
    }
}

// (Re-)initialisation at given fields.  Default: every lattice at its
// equilibrium (Sec. 3.1-3.4, p = 0), the phi populations carrying the first
// moment of the central-difference gradient.  KEEP_FLOW: the flow lattice is
// left as it is and its velocity (at the new phi) enters the C and theta
// equilibria.  KEEP_NONEQ: the phi, C and H populations keep their
// non-equilibrium parts (each moves by the change of its equilibrium, and the
// phi first moment by the change of the central-difference term), and the
// time derivatives carry over at interior nodes.
template <class CF, bool NS, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_set_fields(const KParams kp, const InitFields in,
                                                      typename CF::S* __restrict__ pop,
                                                      typename CF::S* __restrict__ flow,
                                                      typename CF::H* __restrict__ hist) {
    using HT = typename CF::H;
    int x, y;
    if (!node_of_thread(kp, x, y)) return;
    const size_t P = (size_t)kp.plane;
    const size_t idx = (size_t)y * kp.nx + x;
    const bool keep_flow = NS && (in.flags & KEEP_FLOW);
    const bool keep_neq = (in.flags & KEEP_NONEQ) != 0;
    const double phi = in.phi[idx];
    double gx, gy, Vx, Vy;
    cd_gradient<WALLS>(kp, in.phi, x, y, gx, gy);
    phi_first_moment(kp, gx, gy, Vx, Vy);
    const double k = kp.k;
    double C = in.C ? in.C[idx]
                    : (in.c_init_U ? 0.5 * (1.0 + k - (1.0 - k) * phi) * (1.0 + (1.0 - k) * in.U0)
                                   : in.C0);
    double th = in.theta ? in.theta[idx] : in.theta0;
    double ux = in.ux ? in.ux[idx] : in.uin_x;
    double uy = in.uy ? in.uy[idx] : in.uin_y;
    if (!NS) ux = uy = 0.0;
    double hflow[9];
    if constexpr (NS) {
        if (keep_flow || keep_neq)
            for (int i = 0; i < 9; ++i) hflow[i] = ld_pop<double>(flow, i * P + idx, kp.shift[15 + i]);
        if (keep_flow) step_velocity(kp, hflow, phi, ux, uy);
    }
    const double U = (2.0 * C / (1.0 + k - (1.0 - k) * phi) - 1.0) / (1.0 - k);

    // the current state at this node (KEEP_NONEQ)
    double fo[5], no[5], go[5], phio = 0.0, Co = 0.0, Ho = 0.0, uox = 0.0, uoy = 0.0;
    double dVx = 0.0, dVy = 0.0;
    if (keep_neq) {
        for (int i = 0; i < 5; ++i) {
            fo[i] = ld_pop<double>(pop, i * P + idx, kp.shift[i]);
            no[i] = ld_pct<CF, double>(pop, 5 + i, P, idx, kp.shift);
            go[i] = ld_pct<CF, double>(pop, 10 + i, P, idx, kp.shift);
            phio += fo[i];
            Co += no[i];
            Ho += go[i];
        }
        if constexpr (NS) step_velocity(kp, hflow, phio, uox, uoy);
        double gox, goy, Vox, Voy;
        cd_gradient<WALLS>(kp, in.phi_old, x, y, gox, goy);
        phi_first_moment(kp, gox, goy, Vox, Voy);
        dVx = Vx - Vox;
        dVy = Vy - Voy;
    }

    const double w5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
    double e[9], eo[5];
    eq_phi<double>(phi, e);
    if (keep_neq) {
        eq_phi<double>(phio, eo);
        for (int i = 0; i < 5; ++i)
            st_pop(pop, i * P + idx, fo[i] + (e[i] - eo[i]) + 3.0 * w5[i] * (C5X[i] * dVx + C5Y[i] * dVy),
                   kp.shift[i]);
    } else {
        for (int i = 0; i < 5; ++i)
            st_pop(pop, i * P + idx, e[i] + 3.0 * w5[i] * (C5X[i] * Vx + C5Y[i] * Vy), kp.shift[i]);
    }
    eq_solute<double>(C, phi, U, ux, uy, e);
    if (keep_neq) {
        double Uo = (2.0 * Co / (1.0 + k - (1.0 - k) * phio) - 1.0) / (1.0 - k);
        eq_solute<double>(Co, phio, Uo, uox, uoy, eo);
        for (int i = 0; i < 5; ++i) st_pct<CF>(pop, 5 + i, P, idx, no[i] + (e[i] - eo[i]), kp.shift);
    } else {
        for (int i = 0; i < 5; ++i) st_pct<CF>(pop, 5 + i, P, idx, e[i], kp.shift);
    }
    // heat populations carry the velocity of their own step (n_sub_t sub-steps)
    const double ht = kp.n_sub_t;
    eq_heat<double>(th, phi, kp.h_quintic, ux / ht, uy / ht, e);
    if (keep_neq) {
        double tho = Ho + 0.5 * h_of(phio, kp.h_quintic);
        eq_heat<double>(tho, phio, kp.h_quintic, uox / ht, uoy / ht, eo);
        for (int i = 0; i < 5; ++i) st_pct<CF>(pop, 10 + i, P, idx, go[i] + (e[i] - eo[i]), kp.shift);
    } else {
        for (int i = 0; i < 5; ++i) st_pct<CF>(pop, 10 + i, P, idx, e[i], kp.shift);
    }
    double sux = ux, suy = uy;  // the velocity the next step will evaluate
    if constexpr (NS) {
        if (!keep_flow) {
            eq_flow<double>(0.0, 0.0, ux / kp.nsub_d, uy / kp.nsub_d, e);
            for (int i = 0; i < 9; ++i) st_pop(flow, i * P + idx, e[i], kp.shift[15 + i]);
            step_velocity(kp, e, phi, sux, suy);
        }
    }
    // time derivatives: history := new value - (old value - old history)
    if (keep_neq && in.hist_valid && !(WALLS && is_wall(kp, x, y))) {
        const double om = 1.0 - phi * phi;
        const double Q = phi * om - kp.lambda * (th + kp.Mcinf * U) * om * om;
        const double H = th - 0.5 * h_of(phi, kp.h_quintic);
        hist[idx] = HT(phi - (double)hist[idx]);
        hist[P + idx] = HT(Q - (double)hist[P + idx]);
        if constexpr (NS) {
            hist[2 * P + idx] = HT(C * sux - (double)hist[2 * P + idx]);
            hist[3 * P + idx] = HT(C * suy - (double)hist[3 * P + idx]);
            hist[4 * P + idx] = HT(H * sux - (double)hist[4 * P + idx]);
            hist[5 * P + idx] = HT(H * suy - (double)hist[5 * P + idx]);
        }
    }
    // frozen solid: phi of the flow sub-steps, as a main step would leave it
    // (a wall node carries its inward neighbour's value)
    if (in.phi_static) hist[idx] = HT((WALLS && is_wall(kp, x, y)) ? in.phi[inward_idx(kp, x, y)] : phi);
}

// ---------------------------------------------------------------------------
// Observation: macroscopic fields, reductions, tips.
// ---------------------------------------------------------------------------
template <class CF, bool NS, bool WALLS>
__device__ __forceinline__ void node_macros(const KParams& kp, const typename CF::S* __restrict__ pop,
                                            const typename CF::S* __restrict__ flow, int x, int y,
                                            double* m) {
    using T = typename CF::T;
    using S = typename CF::S;
    const size_t P = (size_t)kp.plane;
    const size_t idx = (size_t)y * kp.nx + x;
    const size_t src = (WALLS && is_wall(kp, x, y)) ? inward_idx(kp, x, y) : idx;
    T phi = T(0), C = T(0), H = T(0);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        phi += ld_pop<T>(pop, i * P + src, kp.shift[i]);
        C += ld_pct<CF, T>(pop, 5 + i, P, src, kp.shift);
        H += ld_pct<CF, T>(pop, 10 + i, P, src, kp.shift);
    }
    if constexpr (WALLS && !NS) {
        if (kp.farfield && is_wall(kp, x, y)) {  // the far-field liquid
            phi = T(-1);
            C = T(kp.ff_C);
            H = T(kp.theta0) - T(0.5) * h_of(T(-1), kp.h_quintic);
        }
    }
    T k = T(kp.k);
    if (!kp.use_t) H = T(kp.theta0) - T(0.5) * h_of(phi, kp.h_quintic);  // isothermal
    m[0] = phi;
    m[1] = C;
    m[2] = (T(2) * C / (T(1) + k - (T(1) - k) * phi) - T(1)) / (T(1) - k);
    m[3] = H + T(0.5) * h_of(phi, kp.h_quintic);
    m[4] = m[5] = m[6] = 0.0;
    m[7] = H;
    m[8] = m[9] = 0.0;  // interface force (sub-step units)
    m[10] = m[11] = 0.0;  // f = u_s - u* = -u* (sub-step units)
    if constexpr (NS) {
        T h[9];
        FlowMacro<T> fm;
        if (kp.force) {
            flow_node<T, S, WALLS, true>(kp, flow, x, y, idx, phi, h);
            fm = flow_macro_force(h, phi, kp);
        } else {
            flow_node<T, S, WALLS>(kp, flow, x, y, idx, phi, h);
            fm = flow_macro(h, phi);
        }
        m[4] = kp.nsub_d * fm.ux;
        m[5] = kp.nsub_d * fm.uy;
        m[6] = kp.nsub_d * kp.nsub_d * fm.p;
        m[8] = fm.Fx;
        m[9] = fm.Fy;
        m[10] = -fm.mx;
        m[11] = -fm.my;
    }
}

template <class CF, bool NS, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_fields(const KParams kp,
                                                  const typename CF::S* __restrict__ pop,
                                                  const typename CF::S* __restrict__ flow,
                                                  uint32_t mask, void* __restrict__ out, int f32) {
    int x, y;
    if (!node_of_thread(kp, x, y)) return;
    double m[12];
    node_macros<CF, NS, WALLS>(kp, pop, flow, x, y, m);
    size_t N = (size_t)kp.nx * kp.ny, idx = (size_t)y * kp.nx + x;
    int slot = 0;
    for (int f = 0; f < 7; ++f) {
        if (!(mask & (1u << f))) continue;
        if (f32) ((float*)out)[slot * N + idx] = (float)m[f];
        else ((double*)out)[slot * N + idx] = m[f];
        ++slot;
    }
}

// Block-wide FP64 sum of NR values: wave shuffles, then LDS across the
// four waves.  Result valid in thread 0.
template <int NR> __device__ __forceinline__ void block_sum(double* v) {
    __shared__ double sh[NR][BLOCK / 64];
#pragma unroll
    for (int r = 0; r < NR; ++r)
        for (int off = 32; off > 0; off >>= 1) v[r] += __shfl_xor(v[r], off, 64);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int r = 0; r < NR; ++r) sh[r][wave] = v[r];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int r = 0; r < NR; ++r) {
            double s = 0.0;
            for (int w = 0; w < BLOCK / 64; ++w) s += sh[r][w];
            v[r] = s;
        }
}

static constexpr int NRED = 11;
// partial sums per workgroup: C, H, (1+phi)/2, non-finite, x w, y w, Fx, Fy,
// x Fy - y Fx, and f summed over the nodes with phi > 0 (x, y)
template <class CF, bool NS, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_reduce_partial(const KParams kp,
                                                          const typename CF::S* __restrict__ pop,
                                                          const typename CF::S* __restrict__ flow,
                                                          double* __restrict__ partial) {
    double v[NRED] = {0};
    int x, y;
    if (node_of_thread(kp, x, y)) {
        double m[12];
        node_macros<CF, NS, WALLS>(kp, pop, flow, x, y, m);
        double w = 0.5 * (1.0 + m[0]);
        v[0] = m[1];
        v[1] = m[7];
        v[2] = w;
        bool ok = isfinite(m[0]) && isfinite(m[1]) && isfinite(m[7]);
        if (NS) ok = ok && isfinite(m[4]) && isfinite(m[5]);
        v[3] = ok ? 0.0 : 1.0;
        v[4] = w * x;
        v[5] = w * y;
        v[6] = m[8];
        v[7] = m[9];
        v[8] = x * m[9] - y * m[8];
        if (m[0] > 0.0) {
            v[9] = m[10];
            v[10] = m[11];
        }
    }
    block_sum<NRED>(v);
    if (threadIdx.x == 0)
        for (int r = 0; r < NRED; ++r) partial[(size_t)blockIdx.x * NRED + r] = v[r];
}

// out[0..6] and out[15..16] of the reduction record (see dlb.h)
__global__ __launch_bounds__(BLOCK) void k_reduce_final(const double* __restrict__ partial, int nb,
                                                        long long nodes, double* __restrict__ out) {
    double v[NRED] = {0};
    for (int b = threadIdx.x; b < nb; b += BLOCK)
        for (int r = 0; r < NRED; ++r) v[r] += partial[(size_t)b * NRED + r];
    block_sum<NRED>(v);
    if (threadIdx.x == 0) {
        double cx = v[4] / v[2], cy = v[5] / v[2];
        out[0] = v[0];
        out[1] = v[1];
        out[2] = v[2] / (double)nodes;
        out[3] = v[3];
        out[4] = -v[6];
        out[5] = -v[7];
        // -sum (x - cx) x F = -(sum (x Fy - y Fx) - cx sum Fy + cy sum Fx)
        out[6] = -(v[8] - cx * v[7] + cy * v[6]);
        out[15] = cx;
        out[16] = cy;
        out[17] = -v[9];
        out[18] = -v[10];
    }
}

template <class CF, bool WALLS>
__device__ __forceinline__ double node_phi(const KParams& kp, const typename CF::S* __restrict__ pop,
                                           int x, int y) {
    using T = typename CF::T;
    const size_t P = (size_t)kp.plane;
    if (WALLS && kp.farfield && is_wall(kp, x, y)) return -1.0;
    size_t idx = (WALLS && is_wall(kp, x, y)) ? inward_idx(kp, x, y) : (size_t)y * kp.nx + x;
    T s = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) s += ld_pop<T>(pop, i * P + idx, kp.shift[i]);
    return (double)s;
}

// Bilinear sample of psi = atanh(phi); NaN outside [0, nx-1] x [0, ny-1].
template <class CF, bool WALLS>
__device__ double sample_psi(const KParams& kp, const typename CF::S* __restrict__ pop, double x,
                             double y) {
    // psi = atanh(phi) (phi clamped to |phi| <= 1 - 2^-30) is linear across
    // a tanh interface, so bilinear interpolation of psi is exact for a
    // planar front at any orientation.
    if (!(x >= 0.0 && y >= 0.0 && x <= kp.nx - 1 && y <= kp.ny - 1)) return __builtin_nan("");
    int i0 = (int)floor(x), j0 = (int)floor(y);
    if (i0 > kp.nx - 2) i0 = kp.nx - 2;
    if (j0 > kp.ny - 2) j0 = kp.ny - 2;
    double fx = x - i0, fy = y - j0;
    const double c = 1.0 - 1.0 / 1073741824.0;
    auto psi = [c](double v) { return atanh(v > c ? c : (v < -c ? -c : v)); };
    double p00 = psi(node_phi<CF, WALLS>(kp, pop, i0, j0));
    double p10 = psi(node_phi<CF, WALLS>(kp, pop, i0 + 1, j0));
    double p01 = psi(node_phi<CF, WALLS>(kp, pop, i0, j0 + 1));
    double p11 = psi(node_phi<CF, WALLS>(kp, pop, i0 + 1, j0 + 1));
    return (1.0 - fx) * (1.0 - fy) * p00 + fx * (1.0 - fy) * p10 + (1.0 - fx) * fy * p01 +
           fx * fy * p11;
}

// Tips: one workgroup per arm, one wave per sideways offset w = -3..3; the
// crossing psi_j > 0 >= psi_{j+1} is refined linearly in psi = atanh(phi).
template <class CF, bool WALLS>
__global__ __launch_bounds__(448) void k_tips(const KParams kp, const typename CF::S* __restrict__ pop,
                                              double* __restrict__ out) {
    __shared__ double cross[7];
    const int arm = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double w = (double)(wave - 3);
    const double th = kp.orient + arm * (M_PI / 2.0);
    const double dx = cos(th), dy = sin(th), ex = -sin(th), ey = cos(th);
    long long best = -1;
    // samples j = 0, 1, ... until the first one outside the domain (index J);
    // a crossing needs both samples of the pair inside
    for (long long base = 0;; base += 64) {
        long long j = base + lane;
        double x0 = kp.seed_x + j * dx + w * ex, y0 = kp.seed_y + j * dy + w * ey;
        double x1 = kp.seed_x + (j + 1) * dx + w * ex, y1 = kp.seed_y + (j + 1) * dy + w * ey;
        double v0 = sample_psi<CF, WALLS>(kp, pop, x0, y0);
        double v1 = sample_psi<CF, WALLS>(kp, pop, x1, y1);
        unsigned long long out_mask = __ballot(isnan(v0));
        long long J = out_mask ? base + __ffsll((long long)out_mask) - 1 : base + 64 + 1;
        if (j + 1 < J && v0 > 0.0 && v1 <= 0.0) best = j;
        if (out_mask) break;
    }
    for (int off = 32; off > 0; off >>= 1) {
        long long o = __shfl_xor(best, off, 64);
        best = o > best ? o : best;
    }
    if (lane == 0) {
        double s = __builtin_nan("");
        if (best >= 0) {
            double x0 = kp.seed_x + best * dx + w * ex, y0 = kp.seed_y + best * dy + w * ey;
            double x1 = kp.seed_x + (best + 1) * dx + w * ex;
            double y1 = kp.seed_y + (best + 1) * dy + w * ey;
            double v0 = sample_psi<CF, WALLS>(kp, pop, x0, y0);
            double v1 = sample_psi<CF, WALLS>(kp, pop, x1, y1);
            s = best + v0 / (v0 - v1);
        }
        cross[wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double Sx = 0, Sy = 0, Sxx = 0, Sxy = 0;
        int n = 0;
        for (int k = 0; k < 7; ++k) {
            double c = cross[k];
            if (isnan(c)) continue;
            double X = (double)((k - 3) * (k - 3));
            Sx += X;
            Sy += c;
            Sxx += X * X;
            Sxy += X * c;
            ++n;
        }
        double rho = __builtin_nan("");
        if (n >= 3) {
            double den = n * Sxx - Sx * Sx;
            if (den != 0.0) {
                double B = (n * Sxy - Sx * Sy) / den;
                if (B < 0.0) rho = -1.0 / (2.0 * B);
            }
        }
        out[7 + arm] = cross[3];
        out[11 + arm] = rho;
    }
}

// ---------------------------------------------------------------------------
// Equilibrium check entry point and bandwidth calibration copy.
// ---------------------------------------------------------------------------
__global__ void k_equilibria(long long n, const double* __restrict__ in, double* __restrict__ out,
                             int quintic) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* m = in + 8 * i;
    double* o = out + 24 * i;
    eq_phi<double>(m[0], o);
    eq_solute<double>(m[1], m[0], m[2], m[4], m[5], o + 5);
    eq_heat<double>(m[3], m[0], quintic, m[4], m[5], o + 10);
    eq_flow<double>(m[7], m[6], m[4], m[5], o + 15);
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                              size_t n) {
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace dlb
