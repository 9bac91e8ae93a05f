// lattice.h -- device-side lattice arithmetic of the diffuse-interface MRT
// lattice Boltzmann method (Zhan et al., arXiv:2209.01444) for gfx950.
//
// Everything here works in moment space with the closed forms of the
// Appendix B transforms: the D2Q5 lattices keep (m0, m1x, m1y) live and relax
// the second moments fully (s0 = s2 = 1, Sec. 4 preamble); the D2Q9 flow
// lattice relaxes the raw moments (1, cx, cy, cx^2, cy^2, cxcy, cx^2cy,
// cxcy^2, cx^2cy^2) with S = diag(1, 1, 1, s2, s2, s2, 1, 1, 1).
//
// Velocity order (columns of M, Appendix B):
//   D2Q5: (0,0) (1,0) (0,1) (-1,0) (0,-1)
//   D2Q9: the same, then (1,1) (-1,1) (-1,-1) (1,-1)
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace dlb {

// Kernel-side parameters, passed by value.  Derived quantities are filled in
// on the host from dlb_params (see make_kparams in dlb.hip).
struct KParams {
    int nx, ny;
    long long plane;        // elements per SoA plane (>= nx*ny, 64-element multiple)
    int n_sub, h_quintic, grad_iters, walls;
    int use_t;              // 0: isothermal, theta = theta0 (no heat lattice)
    double theta0;
    int nbx, nby, nblocks;  // tile grid of the node kernels
    double W0, W2t;         // W0, W0^2/tau0
    double inv_tau0, eps4, co, so;
    double lambda, Mcinf, k, invD, s1c, s1t, s2u, jat;  // jat = W0/(2 sqrt 2)
    double nsub_d, uin_x_sub, uin_y_sub, grad_tol2;
    double seed_R, seed_x, seed_y, noise_amp, orient;
    float shift[24];        // storage shifts (rest-state populations) for 16-bit storage
    // row shift and tile rows of the wave-row fused tiles [8 / 12 waves][K = 3 / 5];
    // tbw_tall: the single-solver launch takes the 12-wave tile
    int tbw_dy[2][2], tbw_nby[2][2], tbw_tall;
    int grad_stencil;           // 1: grad phi from the nine-point stencil of the plane phin
    const void* phin;           // phi at time t per node (history type), grad_stencil only
    int n_sub_t;                // heat sub-steps per main step (1: within k_pct)
    void* aux;                  // u, d_t(Hu) of time t (4 planes, history type), n_sub_t > 1 only
    int farfield;               // walls hold the far-field liquid (flow lattice off)
    double ff_C, ff_U;          // far-field C and U (phi = -1)
    int force;                  // external force / varphi on: the _force kernels run
    double fx_sub, fy_sub;      // external force per flow sub-step (F / n_sub^2)
    double varphi, kpf;         // varphi and 3 varphi K (pressure term, times 1/cs^2)
};

// node kernels of a single solver: one row segment of 256 nodes per
// workgroup (longer contiguous runs of the push-streamed stores than 64 x 4:
// the phi/C/theta kernel 2-6% faster, same values)
static constexpr int TILE_X = 256;
static constexpr int TILE_Y = 1;
static constexpr int TILE_X_LOG2 = 8;
static constexpr int BLOCK = TILE_X * TILE_Y;
static_assert((1 << TILE_X_LOG2) == TILE_X, "tile width");
static constexpr double GRAD_GUARD = 1e-12;

// ---------------------------------------------------------------------------
// Storage codecs.  16-bit formats hold shifts from rest-state populations.
// ---------------------------------------------------------------------------
template <class S> struct Prec;
template <> struct Prec<double> { using T = double; static constexpr bool half = false; };
template <> struct Prec<float> { using T = float; static constexpr bool half = false; };
template <> struct Prec<__half> { using T = float; static constexpr bool half = true; };
template <> struct Prec<__hip_bfloat16> { using T = float; static constexpr bool half = true; };

__device__ __forceinline__ double ld_raw(const double* p, size_t i) { return p[i]; }
__device__ __forceinline__ float ld_raw(const float* p, size_t i) { return p[i]; }
__device__ __forceinline__ float ld_raw(const __half* p, size_t i) { return __half2float(p[i]); }
__device__ __forceinline__ float ld_raw(const __hip_bfloat16* p, size_t i) {
    return __bfloat162float(p[i]);
}
__device__ __forceinline__ void st_raw(double* p, size_t i, double v) { p[i] = v; }
__device__ __forceinline__ void st_raw(float* p, size_t i, float v) { p[i] = v; }
__device__ __forceinline__ void st_raw(__half* p, size_t i, float v) { p[i] = __float2half_rn(v); }
__device__ __forceinline__ void st_raw(__hip_bfloat16* p, size_t i, float v) {
    p[i] = __float2bfloat16(v);
}

// Load a population as compute type T / store one from T.
template <class T, class S>
__device__ __forceinline__ T ld_pop(const S* p, size_t i, float shift) {
    if constexpr (Prec<S>::half) return T(ld_raw(p, i) + shift);
    else return T(ld_raw(p, i));
}
template <class S, class T>
__device__ __forceinline__ void st_pop(S* p, size_t i, T v, float shift) {
    using N = typename Prec<S>::T;
    if constexpr (Prec<S>::half) st_raw(p, i, N(v) - shift);
    else st_raw(p, i, N(v));
}

// Precision configurations: storage type S, arithmetic type T, history
// storage type H, storage type SC of the solute and heat populations (S
// except in mixed storage).
template <class S_, class T_, class H_, class SC_ = S_> struct Cfg {
    using S = S_;
    using T = T_;
    using H = H_;
    using SC = SC_;
};
using CfgF64 = Cfg<double, double, double>;
using CfgF32 = Cfg<float, float, float>;
using CfgF32M = Cfg<float, double, float>;  // FP32 storage, FP64 arithmetic
using CfgF16 = Cfg<__half, float, float>;
using CfgBF16 = Cfg<__hip_bfloat16, float, float>;
// mixed: phi and flow populations as FP16 shifts, solute and heat FP32
using CfgF16M = Cfg<__half, float, float, float>;

// Arithmetic of the phi/C/theta kernels (and of the field and tip readers).
// With FP32 storage they compute in FP64: the supersaturation U magnifies the
// rounding of phi sevenfold in the solid (the factor 1/(1 + k - (1 - k) phi)),
// and FP64 here costs about 2% of that kernel's time, since the FP64 and the
// non-packed FP32 vector rates are equal; the flow kernels keep FP32.
template <class CF> struct PctArith { using type = CF; };
template <> struct PctArith<CfgF32> { using type = CfgF32M; };
template <> struct PctArith<CfgF16M> { using type = Cfg<__half, double, float, float>; };

// Population j (0-14) of the phi/C/H block of a population buffer at node
// index idx: the phi planes (j < 5) hold S, the C and H planes CF::SC, all
// planes P elements long.  With SC = S this is plane j, element idx.
template <class CF, class T>
__device__ __forceinline__ T ld_pct(const typename CF::S* pop, int j, size_t P, size_t idx, const float* shift) {
    if (j < 5) return ld_pop<T>(pop, j * P + idx, shift[j]);
    const typename CF::SC* c = reinterpret_cast<const typename CF::SC*>(pop + 5 * P);
    return ld_pop<T>(c, (j - 5) * P + idx, shift[j]);
}
template <class CF, class T>
__device__ __forceinline__ void st_pct(typename CF::S* pop, int j, size_t P, size_t idx, T v, const float* shift) {
    if (j < 5) {
        st_pop(pop, j * P + idx, v, shift[j]);
        return;
    }
    typename CF::SC* c = reinterpret_cast<typename CF::SC*>(pop + 5 * P);
    st_pop(c, (j - 5) * P + idx, v, shift[j]);
}

// ---------------------------------------------------------------------------
// Node geometry.  Workgroups are TILE_X x TILE_Y tiles; the linear workgroup id is
// remapped so each of the 8 XCDs (which receive ids round-robin) walks a
// contiguous band of rows and keeps the y-neighbour rows in its own L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    int q = nb >> 3, r = nb & 7;
    int xcd = bid & 7, slot = bid >> 3;
    int base = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;
    return base + slot;
}

__device__ __forceinline__ bool node_of_thread(const KParams& kp, int& x, int& y) {
    int t = xcd_remap(blockIdx.x, kp.nblocks);
    int bx = t % kp.nbx, by = t / kp.nbx;
    x = bx * TILE_X + (threadIdx.x & (TILE_X - 1));
    y = by * TILE_Y + (threadIdx.x >> TILE_X_LOG2);
    return x < kp.nx && y < kp.ny;
}

__device__ __forceinline__ bool is_wall(const KParams& kp, int x, int y) {
    return x == 0 || y == 0 || x == kp.nx - 1 || y == kp.ny - 1;
}
__device__ __forceinline__ size_t inward_idx(const KParams& kp, int x, int y) {
    int xf = x < 1 ? 1 : (x > kp.nx - 2 ? kp.nx - 2 : x);
    int yf = y < 1 ? 1 : (y > kp.ny - 2 ? kp.ny - 2 : y);
    return (size_t)yf * kp.nx + xf;
}

// ---------------------------------------------------------------------------
// Equilibria in the documented evaluation order (no contraction), shared by
// initialisation, wall rebuilding and the equilibrium check entry point.
// ---------------------------------------------------------------------------
template <class T> __device__ __forceinline__ T h_of(T phi, int quintic) {
#pragma clang fp contract(off)
    if (!quintic) return phi;
    T p2 = phi * phi;
    return T(15.0) * (phi - T(2.0) * phi * p2 / T(3.0) + phi * p2 * p2 / T(5.0)) / T(8.0);
}

// f_i^eq = w_i phi (Sec. 3.1)
template <class T> __device__ void eq_phi(T phi, T* o) {
#pragma clang fp contract(off)
    const T w0 = T(1.0) / T(3.0), w1 = T(1.0) / T(6.0);
    o[0] = w0 * phi;
    o[1] = w1 * phi; o[2] = w1 * phi; o[3] = w1 * phi; o[4] = w1 * phi;
}

// n^eq (Sec. 3.2)
template <class T> __device__ void eq_solute(T C, T phi, T U, T ux, T uy, T* o) {
#pragma clang fp contract(off)
    const T w0 = T(1.0) / T(3.0), w1 = T(1.0) / T(6.0);
    T q = T(0.5) * (T(1.0) - phi);
    T qU = q * U;
    T Cux = C * ux, Cuy = C * uy;
    o[0] = C + (w0 - T(1.0)) * qU;
    o[1] = w1 * qU + w1 * (T(3.0) * Cux);
    o[2] = w1 * qU + w1 * (T(3.0) * Cuy);
    o[3] = w1 * qU + w1 * (T(3.0) * (-Cux));
    o[4] = w1 * qU + w1 * (T(3.0) * (-Cuy));
}

// g^eq (Sec. 3.3)
template <class T> __device__ void eq_heat(T theta, T phi, int quintic, T ux, T uy, T* o) {
#pragma clang fp contract(off)
    const T w0 = T(1.0) / T(3.0), w1 = T(1.0) / T(6.0);
    T hp = h_of(phi, quintic);
    T H = theta - T(0.5) * hp;
    T Hux = H * ux, Huy = H * uy;
    o[0] = w0 * theta - T(0.5) * hp;
    o[1] = w1 * theta + w1 * (T(3.0) * Hux);
    o[2] = w1 * theta + w1 * (T(3.0) * Huy);
    o[3] = w1 * theta + w1 * (T(3.0) * (-Hux));
    o[4] = w1 * theta + w1 * (T(3.0) * (-Huy));
}

// h^eq (Sec. 3.4).  rho0 = 0 gives the shifted form the solver stores.
template <class T> __device__ void eq_flow(T rho0, T p, T ux, T uy, T* o) {
#pragma clang fp contract(off)
    const T w0 = T(4.0) / T(9.0), w1 = T(1.0) / T(9.0), w2 = T(1.0) / T(36.0);
    T uu = ux * ux + uy * uy;
    T cu[9] = {T(0.0), ux, uy, -ux, -uy, ux + uy, -ux + uy, -ux + -uy, ux + -uy};
    o[0] = ((w0 - T(1.0)) * (T(3.0) * p) + rho0) +
           w0 * (T(3.0) * cu[0] + T(4.5) * cu[0] * cu[0] - T(1.5) * uu);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        T w = i < 5 ? w1 : w2;
        o[i] = w * (T(3.0) * p) + w * (T(3.0) * cu[i] + T(4.5) * cu[i] * cu[i] - T(1.5) * uu);
    }
}

// ---------------------------------------------------------------------------
// Anisotropy (Sec. 2), 2-D closed form in the crystal frame:
//   a_s = 1 - 3e + 4e (g'x^4 + g'y^4)/|g|^4
//   N'  = 16 e a_s / |g|^4 (g'x g'y^2 (g'x^2 - g'y^2), g'y g'x^2 (g'y^2 - g'x^2))
// with g' = R(-orient) g and N = R(orient) N'.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void anisotropy(const KParams& kp, T gx, T gy, T& a, T& Nx, T& Ny) {
    const T co = T(kp.co), so = T(kp.so), e = T(kp.eps4);
    T px = co * gx + so * gy, py = -so * gx + co * gy;
    T px2 = px * px, py2 = py * py, g2 = px2 + py2;
    T inv = T(1) / (g2 * g2);
    a = T(1) - T(3) * e + T(4) * e * (px2 * px2 + py2 * py2) * inv;
    T c = T(16) * e * a * inv;
    T nxp = c * px * py2 * (px2 - py2);
    T nyp = c * py * px2 * (py2 - px2);
    Nx = co * nxp - so * nyp;
    Ny = so * nxp + co * nyp;
}

// Local gradient of Sec. 3.1,
//   grad phi = -3 s1(a_s) (m1 + W0^2 N / tau0),  s1 = 1/(3 a_s^2 W0^2/tau0 + 1/2),
// solved by fixed-point iteration from the isotropic guess, with the bulk
// guard |g|^2 < 1e-12 -> g = 0, a_s = 1, N = 0.
template <class T>
__device__ __forceinline__ void local_gradient(const KParams& kp, T m1x, T m1y, T& gx, T& gy, T& a,
                                               T& Nx, T& Ny) {
    const T W2t = T(kp.W2t);
    T s1 = T(1) / (T(3) * W2t + T(0.5));
    gx = T(-3) * s1 * m1x;
    gy = T(-3) * s1 * m1y;
    a = T(1);
    Nx = Ny = T(0);
    const T tol2 = T(kp.grad_tol2);
    for (int it = 0; it < kp.grad_iters; ++it) {
        if (gx * gx + gy * gy < T(GRAD_GUARD)) break;
        anisotropy(kp, gx, gy, a, Nx, Ny);
        s1 = T(1) / (T(3) * a * a * W2t + T(0.5));
        T nx = T(-3) * s1 * (m1x + W2t * Nx);
        T ny = T(-3) * s1 * (m1y + W2t * Ny);
        T d2 = (nx - gx) * (nx - gx) + (ny - gy) * (ny - gy);
        gx = nx;
        gy = ny;
        if (d2 <= tol2 * (gx * gx + gy * gy)) break;
    }
    if (gx * gx + gy * gy < T(GRAD_GUARD)) {
        gx = gy = T(0);
        a = T(1);
        Nx = Ny = T(0);
    } else {
        anisotropy(kp, gx, gy, a, Nx, Ny);
    }
}

// ---------------------------------------------------------------------------
// Flow lattice (Sec. 3.4), sub-step units, h_0 stored shifted by -rho0.
// ---------------------------------------------------------------------------
template <class T> struct FlowMacro {
    T mx, my;   // u* = sum c_i h_i
    T ux, uy;   // u = u* + [1 - q(phi)] f / 2,  f = -u* (u_s = 0, dt' = 1)
    T Fx, Fy;   // [1 - q(phi)] f
    T p;        // cs^2/(1-w0) (sum_{i>0} h_i - w0 |u|^2 / (2 cs^2))
};

template <class T> __device__ __forceinline__ FlowMacro<T> flow_macro(const T* h, T phi) {
    FlowMacro<T> m;
    T d57 = h[5] - h[7], d68 = h[6] - h[8];
    m.mx = (h[1] - h[3]) + (d57 - d68);
    m.my = (h[2] - h[4]) + (d57 + d68);
    T rest = (h[1] + h[2]) + (h[3] + h[4]) + ((h[5] + h[6]) + (h[7] + h[8]));
    T solid = T(0.5) * (T(1) + phi);  // 1 - q(phi)
    m.Fx = -solid * m.mx;
    m.Fy = -solid * m.my;
    m.ux = m.mx + T(0.5) * m.Fx;
    m.uy = m.my + T(0.5) * m.Fy;
    m.p = T(0.6) * (rest - T(2.0 / 3.0) * (m.ux * m.ux + m.uy * m.uy));
    return m;
}

// The same with the external force F of Sec. 3.4 (sub-step units):
// u* = sum c h + F/2, and p gains varphi K u.F / cs^2.
template <class T>
__device__ __forceinline__ FlowMacro<T> flow_macro_force(const T* h, T phi, const KParams& kp) {
#pragma clang fp contract(off)
    FlowMacro<T> m;
    const T Fx = T(kp.fx_sub), Fy = T(kp.fy_sub);
    T d57 = h[5] - h[7], d68 = h[6] - h[8];
    m.mx = ((h[1] - h[3]) + (d57 - d68)) + T(0.5) * Fx;
    m.my = ((h[2] - h[4]) + (d57 + d68)) + T(0.5) * Fy;
    T rest = (h[1] + h[2]) + (h[3] + h[4]) + ((h[5] + h[6]) + (h[7] + h[8]));
    T solid = T(0.5) * (T(1) + phi);  // 1 - q(phi)
    m.Fx = -solid * m.mx;
    m.Fy = -solid * m.my;
    m.ux = m.mx + T(0.5) * m.Fx;
    m.uy = m.my + T(0.5) * m.Fy;
    m.p = T(0.6) * ((rest - T(2.0 / 3.0) * (m.ux * m.ux + m.uy * m.uy)) + T(kp.kpf) * (m.ux * Fx + m.uy * Fy));
    return m;
}

// Per-node factors of the flow collision for the frozen phi of the main
// step: with 1 - q(phi) = (1 + phi)/2 and f = -u*, the velocity is
// u = u* (3 - phi)/4 and the relaxed first moment u + F/2 = u* (1 - phi)/2.
template <class T> struct FlowCoef {
    T cu, c1;
};
template <class T> __device__ __forceinline__ FlowCoef<T> flow_coef(T phi) {
    return {(T(3) - phi) * T(0.25), (T(1) - phi) * T(0.5)};
}

template <class T> __device__ __forceinline__ T fmadd(T a, T b, T c) {
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

// x/3 with 1/3 = 21/64 + 1/192: the product by 21/64 is exact inside the
// fused multiply-add and the rounding of 1/192 weighs 1/64 of the result,
// so x/3 is within one rounding of its correctly rounded value.  A rounded
// 1/3 (FP32: 3e-8 high) is the same for every node and sub-step; scaling the
// momentum into the third-order moments by it left the FP32 velocity 15x and
// the pressure 7x further from FP64 after 30000 flow sub-steps.
template <class T> __device__ __forceinline__ T third(T x) {
    return fmadd(x, T(21.0 / 64.0), x * T(1.0 / 192.0));
}

// One MRT collision (Sec. 3.4, Appendix B transform); returns post-collision
// populations (shifted h_0).  Moments share their partial sums; the inverse
// transform is written with the halved and quartered moment combinations:
// the x-links get (m3' - m8')/2 +- (m1 - m7')/2 and the diagonals
// (+-m5' +- m7' + m8' +- m6')/4.  A rounded constant must not scale a
// conserved or slowly relaxing quantity, or its rounding compounds every
// sub-step (FP32: a relative 3e-8 per sub-step is 5e-4 after 15000 of them):
// the momentum keeps m1 = (m1 - m7') + m7' exactly as the inverse transform
// writes it (not 3 (m1/3)); m8' = (p + |u|^2)/3 is formed as
// 2p + |u|^2 - sum_{i>0} h_i, the same number by the definition of p, so that
// sum_{i>0} h_i (the pressure) changes in a collision only by
// (s2 - 1)(2p + |u|^2 - m3 - m4), in which the rounding of p's 3/5 enters
// once more scaled by s2 - 1 (see p below); the third-order moments take
// m1/3 and m2/3 through third().  Fused multiply-adds are spelled
// out and nothing else is contracted, so every kernel that inlines this
// rounds alike.
template <class T, bool LIQUID = false>
__device__ __forceinline__ void flow_collide(const T* h, FlowCoef<T> c, T s2, T* o) {
#pragma clang fp contract(off)
    const T d57 = h[5] - h[7], d68 = h[6] - h[8];
    const T s57 = h[5] + h[7], s68 = h[6] + h[8], e = s57 + s68;
    const T s24 = h[2] + h[4];
    const T mx = (h[1] - h[3]) + (d57 - d68);
    const T my = (h[2] - h[4]) + (d57 + d68);
    const T m3 = (h[1] + h[3]) + e, m4 = s24 + e, m5 = s57 - s68;
    const T rest = m3 + s24;  // sum of h_1 .. h_8
    // in the melt (phi = -1) both factors are exactly 1
    const T ux = LIQUID ? mx : mx * c.cu, uy = LIQUID ? my : my * c.cu;
    const T m1 = LIQUID ? mx : mx * c.c1, m2 = LIQUID ? my : my * c.c1;  // s1 = 1: u + F/2
    const T ux2 = ux * ux, uu = fmadd(uy, uy, ux2);
    // p = 0.6 rest - 0.4 |u|^2 with 0.6 = 0.625 - 0.025: 0.625 is exact and
    // the rounding of 0.025 is 6e-10 of p, against 4e-8 for a rounded 0.6,
    // which would scale the trace of the second moments by (s2 - 1) 1.2 x 4e-8
    // per sub-step
    const T p = fmadd(T(-0.025), rest, fmadd(T(0.625), rest, T(-0.4) * uu));
    const T r2 = T(1) - s2;
    const T n3 = fmadd(s2, p + ux2, r2 * m3);
    const T n4 = fmadd(s2, fmadd(uy, uy, p), r2 * m4);
    const T n5 = fmadd(s2, ux * uy, r2 * m5);
    const T n6 = third(m2), n7 = third(m1);
    const T n8 = fmadd(T(2), p, uu) - rest;
    o[0] = (n8 - n3) - n4;
    const T hn8 = T(-0.5) * n8;
    const T a1 = fmadd(T(0.5), n3, hn8), a2 = fmadd(T(0.5), n4, hn8);
    const T d7 = m1 - n7, d6 = m2 - n6;
    o[1] = fmadd(T(0.5), d7, a1);
    o[3] = fmadd(T(-0.5), d7, a1);
    o[2] = fmadd(T(0.5), d6, a2);
    o[4] = fmadd(T(-0.5), d6, a2);
    const T q6 = T(0.25) * n6, q7 = T(0.25) * n7;
    const T b = fmadd(T(0.25), n8, q6), bc = fmadd(T(0.25), n8, -q6);
    const T t1 = fmadd(T(0.25), n5, q7), t2 = fmadd(T(0.25), n5, -q7);
    o[5] = b + t1;
    o[6] = b - t1;
    o[7] = bc + t2;
    o[8] = bc - t2;
}

// The collision with the external force F and varphi (Sec. 3.4, Appendix
// B): the forcing moments m_F = [0, F + F_b, 2 varphi F_x u, 2 varphi F_y v,
// varphi (F_x v + F_y u), (F + F_b)/3 (y, x), 2 varphi F.u/3], relaxed with
// (I - S/2); s0 = s1 = s3 = s4 = 1 as in flow_collide, same inverse.
template <class T>
__device__ __forceinline__ void flow_collide_force(const T* h, T phi, const KParams& kp, T s2, T* o) {
#pragma clang fp contract(off)
    const FlowMacro<T> m = flow_macro_force(h, phi, kp);
    const T Fx = T(kp.fx_sub), Fy = T(kp.fy_sub), vp = T(kp.varphi);
    const T s57 = h[5] + h[7], s68 = h[6] + h[8], e = s57 + s68;
    const T m3 = (h[1] + h[3]) + e, m4 = (h[2] + h[4]) + e, m5 = s57 - s68;
    const T ux = m.ux, uy = m.uy, p = m.p;
    const T uu = ux * ux + uy * uy, uF = ux * Fx + uy * Fy;
    const T r2 = T(1) - s2, g2 = T(1) - T(0.5) * s2;
    const T n3 = (r2 * m3 + s2 * (p + ux * ux)) + g2 * (T(2) * vp * Fx * ux);
    const T n4 = (r2 * m4 + s2 * (p + uy * uy)) + g2 * (T(2) * vp * Fy * uy);
    const T n5 = (r2 * m5 + s2 * (ux * uy)) + g2 * (vp * (Fx * uy + Fy * ux));
    const T m1 = ux + T(0.5) * (Fx + m.Fx), m2 = uy + T(0.5) * (Fy + m.Fy);
    const T n6 = third(m2), n7 = third(m1);
    const T n8 = third((p + uu) + vp * uF);
    o[0] = (n8 - n3) - n4;
    const T hn8 = T(-0.5) * n8;
    const T a1 = T(0.5) * n3 + hn8, a2 = T(0.5) * n4 + hn8;
    const T d7 = m1 - n7, d6 = m2 - n6;
    o[1] = fmadd(T(0.5), d7, a1);
    o[3] = fmadd(T(-0.5), d7, a1);
    o[2] = fmadd(T(0.5), d6, a2);
    o[4] = fmadd(T(-0.5), d6, a2);
    const T q6 = T(0.25) * n6, q7 = T(0.25) * n7;
    const T b = T(0.25) * n8 + q6, bc = T(0.25) * n8 - q6;
    const T t1 = T(0.25) * n5 + q7, t2 = T(0.25) * n5 - q7;
    o[5] = b + t1;
    o[6] = b - t1;
    o[7] = bc + t2;
    o[8] = bc - t2;
}

}  // namespace dlb
