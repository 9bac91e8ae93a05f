// dlb3.hip -- three-dimensional phase-field, solute and heat lattices (D3Q7)
// of the diffuse-interface lattice Boltzmann method (Zhan et al.,
// arXiv:2209.01444) on gfx950, and the C ABI of include/dlb3.h.
//
// D3Q7 with cs^2 = 1/4 (w0 = 1/4, w1..6 = 1/8), S = diag(1, s1, s1, s1, 1, 1,
// 1).  With every rate but the first-order ones equal to 1, a collision keeps
// the equilibrium plus (1 - s1) times the first-moment part of the
// populations, and the first-order auxiliary term G enters as (1 - s1/2) G;
// the first-moment part of populations with first moment m is c_i.m/2 on the
// moving links.  So each lattice's post-collision populations are
//   rest: w0 (zeroth-order part),  +-a: w1 (zeroth-order part) +- b_a
// with b_a collecting the first-order terms, written out below.
//
// Melt flow (D3Q19, periodic): every rate but the six second-moment ones is
// 1, so a collision keeps h^eq + (1 - s2) P2(h - h^eq) + F/2, where P2 maps
// the non-equilibrium second moments Pi_ab back to populations: Pi_aa puts
// -Pi_aa on the rest and +Pi_aa/2 on the two faces along a; Pi_ab (a != b)
// puts +-Pi_ab/4 on the four edges in the ab plane (sign of c_a c_b).
//
// State (caller's buffer): pop[2] (ping-pong), each [nz][21][ny][nx] with the
// layers padded to 64 elements -- the 21 populations (phi 0-6, C 7-13, H
// 14-20) of one z-layer lie together, so a workgroup's loads and stores stay
// within a few megabytes; flow[2] (with use_ns), each [nz][19][ny][nx], h_0
// stored as h_0 - rho0; hist[8][N] (phi, Q, C u, H u of the previous step;
// after the phi/C/theta kernel hist[0] holds phi of time t for the flow
// sub-steps); staging[8] double planes (fields in and out, reduction partials).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "dlb3.h"

namespace dlb3 {

static constexpr int BX = 64, BY = 4;
static constexpr double CS2 = 0.25;
static constexpr double GUARD = 1e-12;

struct K3 {
    int nx, ny, nz, nbx, nby, nb;  // grid, tiles per layer in x and y, workgroups
    long long plane;  // elements per history / staging plane (>= N, 64-multiple)
    long long lp;     // elements per population layer (>= nx ny, 64-multiple)
    int use_t, h_quintic, grad_iters;
    double W2t, inv_tau0, eps4, lambda, Mcinf, k, invD, s1c, s1t, jat, grad_tol2, theta0;
    double nsub_d, s2u;  // flow sub-steps per main step, flow relaxation rate
    double uin[3];       // inlet velocity per sub-step (walls)
    float shift[21];     // 16-bit storage: rest-state value of each D3Q7 population
};

// Storage and arithmetic: FP64 and FP32 store what they compute; FP16 and
// BF16 store the difference from the far-field rest state (shift) and
// compute in FP32.  Flow populations are stored with h_0 - rho0, whose rest
// state is zero.
template <class S> struct Arith3 { using T = S; };
template <> struct Arith3<__half> { using T = float; };
template <> struct Arith3<__hip_bfloat16> { using T = float; };
__device__ __forceinline__ double ld3(const double* p, size_t i, float) { return p[i]; }
__device__ __forceinline__ float ld3(const float* p, size_t i, float) { return p[i]; }
__device__ __forceinline__ float ld3(const __half* p, size_t i, float sh) { return __half2float(p[i]) + sh; }
__device__ __forceinline__ float ld3(const __hip_bfloat16* p, size_t i, float sh) { return __bfloat162float(p[i]) + sh; }
__device__ __forceinline__ void st3(double* p, size_t i, double v, float) { p[i] = v; }
__device__ __forceinline__ void st3(float* p, size_t i, float v, float) { p[i] = v; }
__device__ __forceinline__ void st3(__half* p, size_t i, float v, float sh) { p[i] = __float2half(v - sh); }
__device__ __forceinline__ void st3(__hip_bfloat16* p, size_t i, float v, float sh) { p[i] = __float2bfloat16(v - sh); }

// D3Q19 links: rest, faces +x +y +z -x -y -z, edges (xy) ++ -- +- -+, (xz) ++ -- +- -+, (yz) ++ -- +- -+
static constexpr int EX19[19] = {0, 1, 0, 0, -1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static constexpr int EY19[19] = {0, 0, 1, 0, 0, -1, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static constexpr int EZ19[19] = {0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// Workgroups are dispatched round-robin over the 8 XCDs; each XCD takes a
// contiguous range of tiles (a band of z-layers), so the z-neighbour layers
// a node pushes into and re-reads stay in that XCD's L2.
__device__ __forceinline__ int xcd_order3(int bid, int nb) {
    const int q = nb >> 3, r = nb & 7, xcd = bid & 7, slot = bid >> 3;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + slot;
}
__device__ __forceinline__ bool node3(const K3& kp, int& x, int& y, int& z) {
    const int t = xcd_order3((int)blockIdx.x, kp.nb);
    const int nxy = kp.nbx * kp.nby;
    z = t / nxy;
    const int rem = t - z * nxy;
    x = (rem % kp.nbx) * BX + (int)threadIdx.x;
    y = (rem / kp.nbx) * BY + (int)threadIdx.y;
    return x < kp.nx && y < kp.ny;
}
__device__ __forceinline__ size_t id3(const K3& kp, int x, int y, int z) {
    return ((size_t)z * kp.ny + y) * kp.nx + x;
}
// Address of population 0 of node (x, y, z); population q is q * lp further.
__device__ __forceinline__ size_t base3(const K3& kp, int x, int y, int z) {
    return (size_t)z * 21 * (size_t)kp.lp + (size_t)y * kp.nx + x;
}
// Address of flow population 0 of node (x, y, z) ([nz][19][ny][nx] layers).
__device__ __forceinline__ size_t fbase3(const K3& kp, int x, int y, int z) {
    return (size_t)z * 19 * (size_t)kp.lp + (size_t)y * kp.nx + x;
}
__device__ __forceinline__ bool is_wall3(const K3& kp, int x, int y, int z) {
    return x == 0 || y == 0 || z == 0 || x == kp.nx - 1 || y == kp.ny - 1 || z == kp.nz - 1;
}
__device__ __forceinline__ int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }
__device__ __forceinline__ size_t inward3(const K3& kp, int x, int y, int z) {
    return base3(kp, clampi(x, 1, kp.nx - 2), clampi(y, 1, kp.ny - 2), clampi(z, 1, kp.nz - 2));
}
__device__ __forceinline__ size_t inward_f3(const K3& kp, int x, int y, int z) {
    return fbase3(kp, clampi(x, 1, kp.nx - 2), clampi(y, 1, kp.ny - 2), clampi(z, 1, kp.nz - 2));
}
__device__ __forceinline__ size_t inward_id3(const K3& kp, int x, int y, int z) {
    return id3(kp, clampi(x, 1, kp.nx - 2), clampi(y, 1, kp.ny - 2), clampi(z, 1, kp.nz - 2));
}

// D3Q19 flow equilibrium with h_0 shifted by -rho0 (Sec. 3.4, cs^2 = 1/3).
template <class T> __device__ __forceinline__ T heq19(int i, T p, const T* u) {
    const int ax = EX19[i], ay = EY19[i], az = EZ19[i];
    const int nn = ax * ax + ay * ay + az * az;
    const T w = nn == 0 ? T(1.0 / 3.0) : (nn == 1 ? T(1.0 / 18.0) : T(1.0 / 36.0));
    const T cu = T(ax) * u[0] + T(ay) * u[1] + T(az) * u[2];
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T sig = i == 0 ? T(-2) * p : w * T(3) * p;
    return sig + w * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu);
}

// u and p (sub-step units) of flow populations h at phi: u* = sum c h,
// u = u* (3 - phi)/4, p = (rest - |u|^2/2)/2.
template <class T> __device__ __forceinline__ void flow_up3(const T* h, T phi, T* u, T& p) {
    T m[3] = {T(0), T(0), T(0)}, rest = T(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        rest += h[i];
        m[0] += T(EX19[i]) * h[i];
        m[1] += T(EY19[i]) * h[i];
        m[2] += T(EZ19[i]) * h[i];
    }
    const T fac = (T(3) - phi) * T(0.25);
    u[0] = m[0] * fac;
    u[1] = m[1] * fac;
    u[2] = m[2] * fac;
    p = T(0.5) * (rest - T(0.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
}

// Flow populations of node (x, y, z) at the current sub-step: interior nodes
// load them; wall nodes rebuild them from the inward neighbour by
// non-equilibrium extrapolation (Sec. 4 preamble), h = h_f + h^eq(p_b, u_b)
// - h^eq(p_f, u_f): west face inlet u_b = uin, p_b = p_f; east face u_b =
// u_f with its y, z components zeroed on y, z walls, p_b = 0; y and z faces
// free slip, p_b = p_f.  phi_f: phi of the inward neighbour (a wall node
// carries its neighbour's phi).
template <class S, bool WALLS, class T = typename Arith3<S>::T>
__device__ __forceinline__ void flow_node3(const K3& kp, const S* __restrict__ hin, int x, int y, int z, T phi_f,
                                           T* h) {
    const size_t LP = (size_t)kp.lp;
    if (!WALLS || !is_wall3(kp, x, y, z)) {
        const size_t fb = fbase3(kp, x, y, z);
#pragma unroll
        for (int i = 0; i < 19; ++i) h[i] = ld3(hin, i * LP + fb, 0.0f);
        return;
    }
    const size_t f = inward_f3(kp, x, y, z);
    T hf[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) hf[i] = ld3(hin, i * LP + f, 0.0f);
    T uf[3], pf;
    flow_up3(hf, phi_f, uf, pf);
    const bool yw = y == 0 || y == kp.ny - 1, zw = z == 0 || z == kp.nz - 1;
    T ub[3], pb;
    if (x == 0) {
        ub[0] = T(kp.uin[0]);
        ub[1] = T(kp.uin[1]);
        ub[2] = T(kp.uin[2]);
        pb = pf;
    } else {
        ub[0] = uf[0];
        ub[1] = yw ? T(0) : uf[1];
        ub[2] = zw ? T(0) : uf[2];
        pb = x == kp.nx - 1 ? T(0) : pf;
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) h[i] = hf[i] + (heq19(i, pb, ub) - heq19(i, pf, uf));
}

template <class T> __device__ __forceinline__ T h_of3(T phi, int quintic) {
    if (!quintic) return phi;
    T p2 = phi * phi;
    return T(15) * (phi - T(2) * phi * p2 / T(3) + phi * p2 * p2 / T(5)) / T(8);
}

// Cubic anisotropy (Sec. 2, d = 3): a_s = 1 - 3e + 4e sum g_a^4/|g|^4,
// N_a = 16 e a_s (g_a^3 |g|^2 - g_a sum g_b^4)/|g|^4.
template <class T>
__device__ __forceinline__ void aniso3(T e, const T* g, T& a, T* N) {
    T g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    T P = g[0] * g[0] * g[0] * g[0] + g[1] * g[1] * g[1] * g[1] + g[2] * g[2] * g[2] * g[2];
    T inv = T(1) / (g2 * g2);
    a = T(1) - T(3) * e + T(4) * e * P * inv;
    T c = T(16) * e * a * inv;
#pragma unroll
    for (int d = 0; d < 3; ++d) N[d] = c * (g[d] * g[d] * g[d] * g2 - g[d] * P);
}

// Local gradient of Sec. 3.1 with cs^2 = 1/4: g = -(s1/cs^2)(m1 + W0^2 N/tau0),
// s1 = 1/(a^2 W0^2/(tau0 cs^2) + 1/2), fixed point from the isotropic guess.
template <class T>
__device__ __forceinline__ void local_grad3(const K3& kp, const T* m1, T* g, T& a, T* N) {
    const T W2t = T(kp.W2t), e = T(kp.eps4), tol2 = T(kp.grad_tol2);
    T s1 = T(1) / (T(4) * W2t + T(0.5));
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] = T(-4) * s1 * m1[d];
    a = T(1);
    N[0] = N[1] = N[2] = T(0);
    for (int it = 0; it < kp.grad_iters; ++it) {
        if (g[0] * g[0] + g[1] * g[1] + g[2] * g[2] < T(GUARD)) break;
        aniso3(e, g, a, N);
        s1 = T(1) / (T(4) * a * a * W2t + T(0.5));
        T ng[3], d2 = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ng[d] = T(-4) * s1 * (m1[d] + W2t * N[d]);
            d2 += (ng[d] - g[d]) * (ng[d] - g[d]);
        }
        g[0] = ng[0];
        g[1] = ng[1];
        g[2] = ng[2];
        if (d2 <= tol2 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2])) break;
    }
    if (g[0] * g[0] + g[1] * g[1] + g[2] * g[2] < T(GUARD)) {
        g[0] = g[1] = g[2] = T(0);
        a = T(1);
        N[0] = N[1] = N[2] = T(0);
    } else {
        aniso3(e, g, a, N);
    }
}

// Population-0 address of the destination of a push along axis link i
// (1..6), or -1 (a wall node).
template <bool WALLS>
__device__ __forceinline__ long long dest3(const K3& kp, int x, int y, int z, int i) {
    int d = i <= 3 ? 1 : -1, ax = (i - 1) % 3;
    int X = x + (ax == 0 ? d : 0), Y = y + (ax == 1 ? d : 0), Z = z + (ax == 2 ? d : 0);
    if constexpr (WALLS) {
        if (X < 1 || Y < 1 || Z < 1 || X > kp.nx - 2 || Y > kp.ny - 2 || Z > kp.nz - 2) return -1;
    } else {
        X = X < 0 ? X + kp.nx : (X >= kp.nx ? X - kp.nx : X);
        Y = Y < 0 ? Y + kp.ny : (Y >= kp.ny ? Y - kp.ny : Y);
        Z = Z < 0 ? Z + kp.nz : (Z >= kp.nz ? Z - kp.nz : Z);
    }
    return (long long)base3(kp, X, Y, Z);
}

// One main step at every node: collide phi, C, theta (Secs. 3.1-3.3), push.
template <class S, bool WALLS, bool NS>
__global__ __launch_bounds__(BX* BY) void k3_step(const K3 kp, const S* __restrict__ pin, S* __restrict__ pout,
                                                  const S* __restrict__ hin, typename Arith3<S>::T* __restrict__ hist,
                                                  int hist_valid) {
    using T = typename Arith3<S>::T;
    int x, y, z;
    if (!node3(kp, x, y, z)) return;
    const size_t P = (size_t)kp.plane, LP = (size_t)kp.lp;
    const size_t idx = id3(kp, x, y, z), own = base3(kp, x, y, z);
    const bool wall = WALLS && is_wall3(kp, x, y, z);
    const size_t src = wall ? inward3(kp, x, y, z) : own;
    T f[7], n[7], g[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        f[i] = ld3(pin, i * LP + src, kp.shift[i]);
        n[i] = ld3(pin, (7 + i) * LP + src, kp.shift[7 + i]);
        g[i] = kp.use_t ? ld3(pin, (14 + i) * LP + src, kp.shift[14 + i]) : T(0);
    }
    const T phi = ((((((f[0] + f[1]) + f[2]) + f[3]) + f[4]) + f[5]) + f[6]);
    const T C = ((((((n[0] + n[1]) + n[2]) + n[3]) + n[4]) + n[5]) + n[6]);
    const T k = T(kp.k);
    const T hphi = h_of3(phi, kp.h_quintic);
    const T H = kp.use_t ? ((((((g[0] + g[1]) + g[2]) + g[3]) + g[4]) + g[5]) + g[6]) : T(kp.theta0) - T(0.5) * hphi;
    const T theta = kp.use_t ? H + T(0.5) * hphi : T(kp.theta0);
    const T U = (T(2) * C / (T(1) + k - (T(1) - k) * phi) - T(1)) / (T(1) - k);

    // melt velocity of time t in main-step units: n_sub (3 - phi)/4 u*
    T u[3] = {T(0), T(0), T(0)};
    if constexpr (NS) {
        T h[19];
        flow_node3<S, WALLS>(kp, hin, x, y, z, phi, h);
        T m[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            if (EX19[i]) m[0] += EX19[i] > 0 ? h[i] : -h[i];
            if (EY19[i]) m[1] += EY19[i] > 0 ? h[i] : -h[i];
            if (EZ19[i]) m[2] += EZ19[i] > 0 ? h[i] : -h[i];
        }
        const T fac = T(kp.nsub_d) * (T(3) - phi) * T(0.25);
        u[0] = m[0] * fac;
        u[1] = m[1] * fac;
        u[2] = m[2] * fac;
    }

    const T m1[3] = {f[1] - f[4], f[2] - f[5], f[3] - f[6]};
    T gr[3], a, N[3];
    local_grad3<T>(kp, m1, gr, a, N);
    const T a2 = a * a, inv_a2 = T(1) / a2;
    const T s1 = T(1) / (T(4) * a2 * T(kp.W2t) + T(0.5));

    const T om = T(1) - phi * phi;
    const T Q = phi * om - T(kp.lambda) * (theta + T(kp.Mcinf) * U) * om * om;
    T dQ = T(0), dphi = T(0);
    if (hist_valid) {
        dphi = phi - hist[idx];
        dQ = Q - hist[P + idx];
    }
    hist[idx] = phi;
    hist[P + idx] = Q;
    T dCu[3] = {T(0), T(0), T(0)}, dHu[3] = {T(0), T(0), T(0)};
    if constexpr (NS) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T Cu = C * u[d], Hu = H * u[d];
            if (hist_valid) {
                dCu[d] = Cu - hist[(2 + d) * P + idx];
                dHu[d] = Hu - hist[(5 + d) * P + idx];
            }
            hist[(2 + d) * P + idx] = Cu;
            hist[(5 + d) * P + idx] = Hu;
        }
    }

    // phi: rest w0 (phi + A), links w1 (phi + A) +- [(1 - s1) m1/2 - (1 - s1/2) N/(8 a^2)]
    T pf[7];
    {
        const T A = (Q + T(0.5) * a2 * dQ) * T(kp.inv_tau0);
        const T e = phi + A;
        const T c1 = (T(1) - s1) * T(0.5), cN = (T(1) - T(0.5) * s1) * T(0.125) * inv_a2;
        pf[0] = T(0.25) * e;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T b = c1 * m1[d] - cN * N[d];
            pf[1 + d] = T(0.125) * e + b;
            pf[4 + d] = T(0.125) * e - b;
        }
    }
    // anti-trapping current (Sec. 2)
    T J[3] = {T(0), T(0), T(0)};
    {
        const T gn2 = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
        if (gn2 > T(0)) {
            const T c = -T(kp.jat) * (T(1) + (T(1) - k) * U) * dphi / sqrt(gn2);
            J[0] = c * gr[0];
            J[1] = c * gr[1];
            J[2] = c * gr[2];
        }
    }
    // solute: rest C - (1 - w0) qU, links w1 qU +- [Cu/2 + (1 - s1c)(m1 - Cu)/2 + (1 - s1c/2) V/8],
    // V = d_t(Cu)/cs^2 + U grad q + J/D with grad q = -grad phi/2
    T pn[7];
    {
        const T s1c = T(kp.s1c), qU = T(0.5) * (T(1) - phi) * U;
        const T c1 = (T(1) - s1c) * T(0.5), cV = (T(1) - T(0.5) * s1c) * T(0.125);
        pn[0] = C - T(0.75) * qU;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T Cu = C * u[d];
            const T V = T(4) * dCu[d] + T(-0.5) * U * gr[d] + J[d] * T(kp.invD);
            const T b = T(0.5) * Cu + c1 * ((n[1 + d] - n[4 + d]) - Cu) + cV * V;
            pn[1 + d] = T(0.125) * qU + b;
            pn[4 + d] = T(0.125) * qU - b;
        }
    }
    // heat: rest w0 theta - h/2, links w1 theta +- [Hu/2 + (1 - s1t)(m1 - Hu)/2 + (1 - s1t/2) d_t(Hu)/2]
    T pg[7];
    {
        const T s1t = T(kp.s1t);
        const T c1 = (T(1) - s1t) * T(0.5), cG = (T(1) - T(0.5) * s1t) * T(0.5);
        pg[0] = T(0.25) * theta - T(0.5) * hphi;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T Hu = H * u[d];
            const T b = T(0.5) * Hu + c1 * ((g[1 + d] - g[4 + d]) - Hu) + cG * dHu[d];
            pg[1 + d] = T(0.125) * theta + b;
            pg[4 + d] = T(0.125) * theta - b;
        }
    }
    // push; phi: f(y, t+1) = f(y, t) + (post - f(y, t)) / a_s^2 (collision site's a_s)
    if (!wall) {
        st3(pout, own, f[0] + (pf[0] - f[0]) * inv_a2, kp.shift[0]);
        st3(pout, 7 * LP + own, pn[0], kp.shift[7]);
        if (kp.use_t) st3(pout, 14 * LP + own, pg[0], kp.shift[14]);
    }
#pragma unroll
    for (int i = 1; i < 7; ++i) {
        const long long d = dest3<WALLS>(kp, x, y, z, i);
        if (d < 0) continue;
        const T fold = ld3(pin, i * LP + (size_t)d, kp.shift[i]);
        st3(pout, i * LP + (size_t)d, fold + (pf[i] - fold) * inv_a2, kp.shift[i]);
        st3(pout, (7 + i) * LP + (size_t)d, pn[i], kp.shift[7 + i]);
        if (kp.use_t) st3(pout, (14 + i) * LP + (size_t)d, pg[i], kp.shift[14 + i]);
    }
}

// One melt-flow sub-step (Sec. 3.4, D3Q19, periodic) at the frozen phi of
// time t (hist[0]), push streaming.
template <class S, bool WALLS>
__global__ __launch_bounds__(BX* BY) void k3_flow(const K3 kp, const S* __restrict__ hin, S* __restrict__ hout,
                                                  const typename Arith3<S>::T* __restrict__ phi_t) {
    using T = typename Arith3<S>::T;
    int x, y, z;
    if (!node3(kp, x, y, z)) return;
    const size_t LP = (size_t)kp.lp;
    const T phi = phi_t[id3(kp, x, y, z)];
    T h[19];
    flow_node3<S, WALLS>(kp, hin, x, y, z, phi, h);
    T m[3] = {T(0), T(0), T(0)}, rest = T(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        rest += h[i];
        m[0] += T(EX19[i]) * h[i];
        m[1] += T(EY19[i]) * h[i];
        m[2] += T(EZ19[i]) * h[i];
    }
    const T solid = T(0.5) * (T(1) + phi);  // 1 - q(phi); f = -u*
    T Fb[3], u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Fb[d] = -solid * m[d];
        u[d] = m[d] + T(0.5) * Fb[d];
    }
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T p = T(0.5) * (rest - T(0.5) * uu);  // cs^2/(1 - w0) (rest - w0 |u|^2/(2 cs^2))
    // The parts of the equilibrium and the forcing that carry mass, momentum
    // and pressure are built from one twelfth of p, u and F_b (3 w = 1/6 on
    // the axes is twice 1/12, on the diagonals 1/12), so that they sum back to
    // 2p, u and F_b/2 up to unbiased rounding; weights 1/18 and 1/36 rounded
    // to FP32 would scale them by 1 + 7.5e-9 every sub-step.  1/12 is
    // 21/256 + 1/768: the first exact, the rounding of the second 5e-10 of
    // the result.  h_0^eq closes the mass: minus the sum of the others.
    auto twelfth = [](T v) { return v * T(21.0 / 256.0) + v * T(1.0 / 768.0); };
    const T tp = twelfth(p);
    const T tu[3] = {twelfth(u[0]), twelfth(u[1]), twelfth(u[2])};
    const T tf[3] = {twelfth(Fb[0]), twelfth(Fb[1]), twelfth(Fb[2])};
    T heq[19], Pi[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    T moving = T(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const int ax = EX19[i], ay = EY19[i], az = EZ19[i];
        const int nn = ax * ax + ay * ay + az * az;
        const T w = nn == 1 ? T(1.0 / 18.0) : T(1.0 / 36.0);
        const T cu = T(ax) * u[0] + T(ay) * u[1] + T(az) * u[2];
        const T lin = (T(ax) * tu[0] + T(ay) * tu[1] + T(az) * tu[2]) + tp;  // 3 w (p + c.u) / (nn == 1 ? 2 : 1)
        heq[i] = (nn == 1 ? T(2) * lin : lin) + w * (T(4.5) * cu * cu - T(1.5) * uu);
        moving += heq[i];
        const T dn = h[i] - heq[i];
        Pi[0] += T(ax * ax) * dn;
        Pi[1] += T(ay * ay) * dn;
        Pi[2] += T(az * az) * dn;
        Pi[3] += T(ax * ay) * dn;
        Pi[4] += T(ax * az) * dn;
        Pi[5] += T(ay * az) * dn;
    }
    heq[0] = -moving;
    const T r = T(1) - T(kp.s2u);
    const int xp = x + 1 == kp.nx ? 0 : x + 1, xm = x == 0 ? kp.nx - 1 : x - 1;
    const int yp = y + 1 == kp.ny ? 0 : y + 1, ym = y == 0 ? kp.ny - 1 : y - 1;
    const int zp = z + 1 == kp.nz ? 0 : z + 1, zm = z == 0 ? kp.nz - 1 : z - 1;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const int ax = EX19[i], ay = EY19[i], az = EZ19[i];
        const int nn = ax * ax + ay * ay + az * az;
        // forcing (1 - 1/2) 3 w c.F_b: c.F_b/12 on the axes, half that on the diagonals
        const T cf = T(ax) * tf[0] + T(ay) * tf[1] + T(az) * tf[2];
        T post = heq[i] + (nn == 1 ? cf : T(0.5) * cf);
        if (nn == 0) post += r * -((Pi[0] + Pi[1]) + Pi[2]);
        else if (nn == 1) post += r * T(0.5) * (ax ? Pi[0] : (ay ? Pi[1] : Pi[2]));
        else post += r * T(0.25) * (az == 0 ? T(ax * ay) * Pi[3] : (ay == 0 ? T(ax * az) * Pi[4] : T(ay * az) * Pi[5]));
        int X, Y, Z;
        if constexpr (WALLS) {  // wall destinations are rebuilt when read
            X = x + ax;
            Y = y + ay;
            Z = z + az;
            if (X < 1 || Y < 1 || Z < 1 || X > kp.nx - 2 || Y > kp.ny - 2 || Z > kp.nz - 2) continue;
        } else {
            X = ax > 0 ? xp : (ax < 0 ? xm : x);
            Y = ay > 0 ? yp : (ay < 0 ? ym : y);
            Z = az > 0 ? zp : (az < 0 ? zm : z);
        }
        st3(hout, i * LP + fbase3(kp, X, Y, Z), post, 0.0f);
    }
}

// Spherical seed into a double plane.
__global__ __launch_bounds__(BX* BY) void k3_seed(const K3 kp, double R, double cx, double cy, double cz,
                                                  double W0, double* __restrict__ phi) {
    int x, y, z;
    if (!node3(kp, x, y, z)) return;
    const double dx = x - cx, dy = y - cy, dz = z - cz;
    phi[id3(kp, x, y, z)] = tanh((R - sqrt(dx * dx + dy * dy + dz * dz)) / (sqrt(2.0) * W0));
}

// Equilibrium at the given fields; phi populations with the first moment
// m1 = -(cs^2/s1) grad phi - W0^2 N/tau0 of the isotropic D3Q19 central
// difference of phi (periodic wrap or clamped at walls).
template <class T, bool WALLS, bool NS>
__global__ __launch_bounds__(BX* BY) void k3_set(const K3 kp, const double* __restrict__ phi,
                                                 const double* __restrict__ Cin, const double* __restrict__ thin,
                                                 const double* __restrict__ uxin, const double* __restrict__ uyin,
                                                 const double* __restrict__ uzin, double u0x, double u0y, double u0z,
                                                 int c_init_U, double U0, double C0, T* __restrict__ pop,
                                                 T* __restrict__ flow) {
    using A = typename Arith3<T>::T;
    int x, y, z;
    if (!node3(kp, x, y, z)) return;
    const size_t idx = id3(kp, x, y, z);
    double gd[3] = {0.0, 0.0, 0.0};
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int nnz = (dx != 0) + (dy != 0) + (dz != 0);
                if (nnz == 0 || nnz == 3) continue;
                const double w = nnz == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
                int X = x + dx, Y = y + dy, Z = z + dz;
                if (WALLS) {
                    X = clampi(X, 0, kp.nx - 1);
                    Y = clampi(Y, 0, kp.ny - 1);
                    Z = clampi(Z, 0, kp.nz - 1);
                } else {
                    X = (X + kp.nx) % kp.nx;
                    Y = (Y + kp.ny) % kp.ny;
                    Z = (Z + kp.nz) % kp.nz;
                }
                const double v = phi[id3(kp, X, Y, Z)];
                gd[0] += 3.0 * w * dx * v;
                gd[1] += 3.0 * w * dy * v;
                gd[2] += 3.0 * w * dz * v;
            }
    double m1[3] = {0.0, 0.0, 0.0};
    if (gd[0] * gd[0] + gd[1] * gd[1] + gd[2] * gd[2] >= GUARD) {
        double a, N[3];
        aniso3(kp.eps4, gd, a, N);
        const double s1 = 1.0 / (4.0 * a * a * kp.W2t + 0.5);
        for (int d = 0; d < 3; ++d) m1[d] = -CS2 * gd[d] / s1 - kp.W2t * N[d];
    }
    const double ph = phi[idx];
    const double k = kp.k;
    const double C = Cin ? Cin[idx]
                         : (c_init_U ? 0.5 * (1.0 + k - (1.0 - k) * ph) * (1.0 + (1.0 - k) * U0) : C0);
    const double th = thin ? thin[idx] : kp.theta0;
    const double U = (2.0 * C / (1.0 + k - (1.0 - k) * ph) - 1.0) / (1.0 - k);
    const double qU = 0.5 * (1.0 - ph) * U;
    const double hp = h_of3(ph, kp.h_quintic);
    double u[3] = {0.0, 0.0, 0.0};
    if (NS) {
        u[0] = uxin ? uxin[idx] : u0x;
        u[1] = uyin ? uyin[idx] : u0y;
        u[2] = uzin ? uzin[idx] : u0z;
    }
    const double H = th - 0.5 * hp;
    const size_t LP = (size_t)kp.lp, o = base3(kp, x, y, z);
    st3(pop, o, A(0.25 * ph), kp.shift[0]);
    st3(pop, 7 * LP + o, A(C - 0.75 * qU), kp.shift[7]);
    st3(pop, 14 * LP + o, A(kp.use_t ? 0.25 * th - 0.5 * hp : 0.0), kp.shift[14]);
    for (int d = 0; d < 3; ++d) {
        // w1 c.(C u)/cs^2 = +-(C u)/2 on the D3Q7 links
        st3(pop, (1 + d) * LP + o, A(0.125 * ph + 0.5 * m1[d]), kp.shift[1 + d]);
        st3(pop, (4 + d) * LP + o, A(0.125 * ph - 0.5 * m1[d]), kp.shift[4 + d]);
        st3(pop, (8 + d) * LP + o, A(0.125 * qU + 0.5 * C * u[d]), kp.shift[8 + d]);
        st3(pop, (11 + d) * LP + o, A(0.125 * qU - 0.5 * C * u[d]), kp.shift[11 + d]);
        st3(pop, (15 + d) * LP + o, A(kp.use_t ? 0.125 * th + 0.5 * H * u[d] : 0.0), kp.shift[15 + d]);
        st3(pop, (18 + d) * LP + o, A(kp.use_t ? 0.125 * th - 0.5 * H * u[d] : 0.0), kp.shift[18 + d]);
    }
    if constexpr (NS) {  // flow at p = 0, u' = u/n_sub (h_0 shifted by -rho0)
        const double v[3] = {u[0] / kp.nsub_d, u[1] / kp.nsub_d, u[2] / kp.nsub_d};
        const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const size_t fb = fbase3(kp, x, y, z);
        for (int i = 0; i < 19; ++i) {
            const int nn = EX19[i] * EX19[i] + EY19[i] * EY19[i] + EZ19[i] * EZ19[i];
            const double w = nn == 0 ? 1.0 / 3.0 : (nn == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
            const double cu = EX19[i] * v[0] + EY19[i] * v[1] + EZ19[i] * v[2];
            st3(flow, i * LP + fb, A(w * (3.0 * cu + 4.5 * cu * cu - 1.5 * vv)), 0.0f);
        }
    }
}

template <class S, bool WALLS, bool NS>
__device__ __forceinline__ void macros3(const K3& kp, const S* __restrict__ pop, const S* __restrict__ flow, int x,
                                        int y, int z, double* m) {
    using T = typename Arith3<S>::T;
    const size_t LP = (size_t)kp.lp;
    const size_t src = (WALLS && is_wall3(kp, x, y, z)) ? inward3(kp, x, y, z) : base3(kp, x, y, z);
    T phi = T(0), C = T(0), H = T(0);
    for (int i = 0; i < 7; ++i) {
        phi += ld3(pop, i * LP + src, kp.shift[i]);
        C += ld3(pop, (7 + i) * LP + src, kp.shift[7 + i]);
        if (kp.use_t) H += ld3(pop, (14 + i) * LP + src, kp.shift[14 + i]);
    }
    const T k = T(kp.k);
    const T hp = h_of3(phi, kp.h_quintic);
    if (!kp.use_t) H = T(kp.theta0) - T(0.5) * hp;
    m[0] = phi;
    m[1] = C;
    m[2] = (T(2) * C / (T(1) + k - (T(1) - k) * phi) - T(1)) / (T(1) - k);
    m[3] = H + T(0.5) * hp;
    m[4] = H;
    m[5] = m[6] = m[7] = m[8] = 0.0;
    if constexpr (NS) {  // u = n_sub u' and p = n_sub^2 p' (main-step units)
        T h[19], u[3], p;
        flow_node3<S, WALLS>(kp, flow, x, y, z, phi, h);
        flow_up3(h, phi, u, p);
        m[5] = kp.nsub_d * u[0];
        m[6] = kp.nsub_d * u[1];
        m[7] = kp.nsub_d * u[2];
        m[8] = kp.nsub_d * kp.nsub_d * p;
    }
}

template <class T, bool WALLS, bool NS>
__global__ __launch_bounds__(BX* BY) void k3_fields(const K3 kp, const T* __restrict__ pop, const T* __restrict__ flow,
                                                    double* __restrict__ out) {
    int x, y, z;
    if (!node3(kp, x, y, z)) return;
    double m[9];
    macros3<T, WALLS, NS>(kp, pop, flow, x, y, z, m);
    const size_t N = (size_t)kp.nx * kp.ny * kp.nz, idx = id3(kp, x, y, z);
    for (int j = 0; j < 4; ++j) out[j * N + idx] = m[j];
    for (int j = 0; j < 4; ++j) out[(4 + j) * N + idx] = m[5 + j];
}

// Per-workgroup partial sums: C, H, (1 + phi)/2, non-finite count.
template <class T, bool WALLS>
__global__ __launch_bounds__(BX* BY) void k3_partial(const K3 kp, const T* __restrict__ pop, double* __restrict__ part) {
    __shared__ double sh[4][BX * BY / 64];
    int x, y, z;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (node3(kp, x, y, z)) {
        double m[9];
        macros3<T, WALLS, false>(kp, pop, nullptr, x, y, z, m);
        v[0] = m[1];
        v[1] = m[4];
        v[2] = 0.5 * (1.0 + m[0]);
        v[3] = (isfinite(m[0]) && isfinite(m[1]) && isfinite(m[3])) ? 0.0 : 1.0;
    }
    const int t = threadIdx.y * BX + threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int r = 0; r < 4; ++r)
        for (int off = 32; off > 0; off >>= 1) v[r] += __shfl_xor(v[r], off, 64);
    if (lane == 0)
        for (int r = 0; r < 4; ++r) sh[r][wave] = v[r];
    __syncthreads();
    if (t == 0) {
        const size_t b = blockIdx.x;
        for (int r = 0; r < 4; ++r) {
            double s = 0.0;
            for (int w = 0; w < BX * BY / 64; ++w) s += sh[r][w];
            part[b * 4 + r] = s;
        }
    }
}

// Final FP64 sums of the per-workgroup partials (one workgroup).
__global__ __launch_bounds__(256) void k3_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double sh[4][4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int r = 0; r < 4; ++r) v[r] += part[(size_t)b * 4 + r];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = 0; r < 4; ++r)
        for (int off = 32; off > 0; off >>= 1) v[r] += __shfl_xor(v[r], off, 64);
    if (lane == 0)
        for (int r = 0; r < 4; ++r) sh[r][wave] = v[r];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int r = 0; r < 4; ++r) out[r] = ((sh[r][0] + sh[r][1]) + sh[r][2]) + sh[r][3];
}

// Tips along the six axis directions from the seed node (one thread each).
template <class T, bool WALLS>
__global__ void k3_tips(const K3 kp, const T* __restrict__ pop, int cx, int cy, int cz, double* __restrict__ out) {
    const int arm = threadIdx.x;
    if (arm >= 6) return;
    const int sgn = arm < 3 ? 1 : -1, ax = arm % 3;
    const double lim = 1.0 - 1.0 / 1073741824.0;
    double best = -1.0, prev = 0.0;
    for (int j = 0;; ++j) {
        const int x = cx + (ax == 0 ? sgn * j : 0), y = cy + (ax == 1 ? sgn * j : 0), z = cz + (ax == 2 ? sgn * j : 0);
        if (x < 0 || y < 0 || z < 0 || x >= kp.nx || y >= kp.ny || z >= kp.nz) break;
        double m[9];
        macros3<T, WALLS, false>(kp, pop, nullptr, x, y, z, m);
        double v = m[0] > lim ? lim : (m[0] < -lim ? -lim : m[0]);
        const double ps = atanh(v);
        if (j > 0 && prev > 0.0 && ps <= 0.0) best = (j - 1) + prev / (prev - ps);
        prev = ps;
    }
    out[arm] = best;
}

}  // namespace dlb3

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
using namespace dlb3;

namespace {
thread_local std::string g_err3;
int fail3(int code, const std::string& m) {
    g_err3 = m;
    return code;
}
int hip_fail3(hipError_t e, const char* what) {
    return fail3(DLB3_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Layout3 {
    size_t plane, lp, pop[2], flow[2], hist, stage, total;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int check3(const dlb3_params* p) {
    if (!p) return fail3(DLB3_EINVAL, "null params");
    if (p->nx < 8 || p->ny < 8 || p->nz < 8) return fail3(DLB3_EINVAL, "grid must be at least 8x8x8");
    if (p->nz > 65535) return fail3(DLB3_EINVAL, "nz must be at most 65535");
    if ((double)p->nx * p->ny * p->nz > 2.0e9) return fail3(DLB3_EINVAL, "grid too large");
    if ((double)((p->nx + BX - 1) / BX) * ((p->ny + BY - 1) / BY) * p->nz > 2.0e9)
        return fail3(DLB3_EINVAL, "too many workgroups");
    if (p->precision < DLB3_F64 || p->precision > DLB3_BF16S) return fail3(DLB3_EINVAL, "unknown precision");
    if (p->walls != 0 && p->walls != 1) return fail3(DLB3_EINVAL, "walls must be 0 or 1");
    if (!(p->W0 > 0 && p->tau0 > 0 && p->D > 0 && p->alpha > 0)) return fail3(DLB3_EINVAL, "W0, tau0, D, alpha must be > 0");
    if (!(p->k > 0 && p->k < 1)) return fail3(DLB3_EINVAL, "partition coefficient k must be in (0,1)");
    if (!(p->eps4 >= 0.0 && p->eps4 < 0.2)) return fail3(DLB3_EINVAL, "eps4 must be in [0, 0.2)");
    const double W2t = p->W0 * p->W0 / p->tau0;
    const double rates[3] = {1.0 / (4.0 * (1.0 + p->eps4) * (1.0 + p->eps4) * W2t + 0.5),
                             1.0 / (4.0 * p->D * (1.0 - p->k) + 0.5), 1.0 / (4.0 * p->alpha + 0.5)};
    for (double r : rates)
        if (!(r > 0.0 && r < 2.0)) return fail3(DLB3_EINVAL, "relaxation rate outside (0,2)");
    if (p->use_ns != 0 && p->use_ns != 1) return fail3(DLB3_EINVAL, "use_ns must be 0 or 1");
    if (p->use_ns) {
        if (p->n_sub < 1 || !(p->nu > 0)) return fail3(DLB3_EINVAL, "melt flow needs n_sub >= 1 and nu > 0");
        const double s2 = 1.0 / (3.0 * p->nu / p->n_sub + 0.5);
        if (!(s2 > 0.0 && s2 < 2.0)) return fail3(DLB3_EINVAL, "relaxation rate outside (0,2)");
        const double mach = std::sqrt(p->u0[0] * p->u0[0] + p->u0[1] * p->u0[1] + p->u0[2] * p->u0[2]) /
                            p->n_sub * std::sqrt(3.0);
        if (!(mach <= 0.3)) return fail3(DLB3_EINVAL, "initial Mach number |u0| sqrt(3)/n_sub exceeds 0.3");
    }
    return DLB3_OK;
}

Layout3 layout3(const dlb3_params* p) {
    Layout3 L{};
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    L.plane = (N + 63) & ~size_t(63);
    L.lp = ((size_t)p->nx * p->ny + 63) & ~size_t(63);
    const size_t sb = p->precision == DLB3_F64 ? 8 : (p->precision == DLB3_F32 ? 4 : 2);
    const size_t hb = p->precision == DLB3_F64 ? 8 : 4;  // history in the arithmetic type
    size_t off = 0;
    for (int b = 0; b < 2; ++b) {
        L.pop[b] = off;
        off = align256(off + (size_t)p->nz * 21 * L.lp * sb);
    }
    for (int b = 0; b < 2; ++b) {
        L.flow[b] = off;
        if (p->use_ns) off = align256(off + (size_t)p->nz * 19 * L.lp * sb);
    }
    L.hist = off;
    off = align256(off + (p->use_ns ? 8 : 2) * L.plane * hb);
    L.stage = off;
    off = align256(off + 8 * L.plane * sizeof(double));
    L.total = off;
    return L;
}

// Rest state of the D3Q7 populations (the 16-bit storage shifts): liquid
// phi = -1 with the initial far-field solute and temperature, moving at the
// initial velocity when the melt flows.
void rest_shifts3(const dlb3_params* p, float* sh) {
    const double k = p->k, phi = -1.0;
    const double C = p->c_init_U ? 1.0 + (1.0 - k) * p->U0 : p->C0;
    const double U = (C - 1.0) / (1.0 - k);  // phi = -1: 1 + k - (1 - k) phi = 2
    const double qU = 0.5 * (1.0 - phi) * U, hp = -1.0;  // h(-1) = -1 for both forms
    const double th = p->theta0, H = th - 0.5 * hp;
    sh[0] = (float)(0.25 * phi);
    sh[7] = (float)(C - 0.75 * qU);
    sh[14] = (float)(0.25 * th - 0.5 * hp);
    for (int d = 0; d < 3; ++d) {
        const double u = p->use_ns ? p->u0[d] : 0.0;
        sh[1 + d] = sh[4 + d] = (float)(0.125 * phi);
        sh[8 + d] = (float)(0.125 * qU + 0.5 * C * u);
        sh[11 + d] = (float)(0.125 * qU - 0.5 * C * u);
        sh[15 + d] = (float)(0.125 * th + 0.5 * H * u);
        sh[18 + d] = (float)(0.125 * th - 0.5 * H * u);
    }
}

K3 make_k3(const dlb3_params* p, const Layout3& L) {
    K3 k{};
    k.nx = p->nx;
    k.ny = p->ny;
    k.nz = p->nz;
    k.nbx = (p->nx + BX - 1) / BX;
    k.nby = (p->ny + BY - 1) / BY;
    k.nb = k.nbx * k.nby * p->nz;
    k.plane = (long long)L.plane;
    k.lp = (long long)L.lp;
    k.use_t = p->use_t ? 1 : 0;
    k.h_quintic = p->h_quintic;
    const bool f64 = p->precision == DLB3_F64;
    k.grad_iters = p->grad_iters > 0 ? p->grad_iters : (f64 ? 100 : 20);
    const double tol = p->grad_tol > 0 ? p->grad_tol : (f64 ? 1e-14 : 1e-6);
    k.grad_tol2 = tol * tol;
    k.W2t = p->W0 * p->W0 / p->tau0;
    k.inv_tau0 = 1.0 / p->tau0;
    k.eps4 = p->eps4;
    k.lambda = p->lambda;
    k.Mcinf = p->Mcinf;
    k.k = p->k;
    k.invD = 1.0 / p->D;
    k.s1c = 1.0 / (4.0 * p->D * (1.0 - p->k) + 0.5);
    k.s1t = 1.0 / (4.0 * p->alpha + 0.5);
    k.jat = p->W0 / (2.0 * std::sqrt(2.0));
    k.theta0 = p->theta0;
    k.nsub_d = p->use_ns ? p->n_sub : 1;
    k.s2u = p->use_ns ? 1.0 / (3.0 * p->nu / p->n_sub + 0.5) : 1.0;
    for (int a = 0; a < 3; ++a) k.uin[a] = p->use_ns ? p->u0[a] / p->n_sub : 0.0;
    if (p->precision == DLB3_F16S || p->precision == DLB3_BF16S) rest_shifts3(p, k.shift);
    return k;
}
}  // namespace

struct dlb3_solver {
    dlb3_params p;
    Layout3 L;
    K3 kp;
    char* base;
    hipStream_t stream;
    int cur, fcur, hist_valid;
    dim3 grid, block;
    const void* pop() const { return base + L.pop[cur]; }
    const void* flow() const { return p.use_ns ? base + L.flow[fcur] : nullptr; }
};

template <class T, bool W> static void launch_step(dlb3_solver* s) {
    if (s->p.use_ns) {
        hipLaunchKernelGGL((k3_step<T, W, true>), s->grid, s->block, 0, s->stream, s->kp, (const T*)s->pop(),
                           (T*)(s->base + s->L.pop[1 - s->cur]), (const T*)s->flow(),
                           (typename Arith3<T>::T*)(s->base + s->L.hist), s->hist_valid);
        return;
    }
    hipLaunchKernelGGL((k3_step<T, W, false>), s->grid, s->block, 0, s->stream, s->kp, (const T*)s->pop(),
                       (T*)(s->base + s->L.pop[1 - s->cur]), (const T*)nullptr,
                       (typename Arith3<T>::T*)(s->base + s->L.hist), s->hist_valid);
}
template <class T, bool W> static void launch_flow(dlb3_solver* s) {
    hipLaunchKernelGGL((k3_flow<T, W>), s->grid, s->block, 0, s->stream, s->kp, (const T*)s->flow(),
                       (T*)(s->base + s->L.flow[1 - s->fcur]), (const typename Arith3<T>::T*)(s->base + s->L.hist));
}
template <class T, bool W>
static void launch_set(dlb3_solver* s, const double* phi, const double* C, const double* th, const double* ux,
                       const double* uy, const double* uz) {
    const double* u0 = s->p.u0;
    if (s->p.use_ns) {
        hipLaunchKernelGGL((k3_set<T, W, true>), s->grid, s->block, 0, s->stream, s->kp, phi, C, th, ux, uy, uz, u0[0],
                           u0[1], u0[2], s->p.c_init_U, s->p.U0, s->p.C0, (T*)(s->base + s->L.pop[s->cur]),
                           (T*)(s->base + s->L.flow[s->fcur]));
        return;
    }
    hipLaunchKernelGGL((k3_set<T, W, false>), s->grid, s->block, 0, s->stream, s->kp, phi, C, th, ux, uy, uz, u0[0],
                       u0[1], u0[2], s->p.c_init_U, s->p.U0, s->p.C0, (T*)(s->base + s->L.pop[s->cur]), (T*)nullptr);
}
template <class T, bool W> static void launch_fields(dlb3_solver* s, double* out) {
    if (s->p.use_ns) {
        hipLaunchKernelGGL((k3_fields<T, W, true>), s->grid, s->block, 0, s->stream, s->kp, (const T*)s->pop(),
                           (const T*)s->flow(), out);
        return;
    }
    hipLaunchKernelGGL((k3_fields<T, W, false>), s->grid, s->block, 0, s->stream, s->kp, (const T*)s->pop(),
                       (const T*)nullptr, out);
}
template <class T, bool W> static void launch_partial(dlb3_solver* s, double* part) {
    hipLaunchKernelGGL((k3_partial<T, W>), s->grid, s->block, 0, s->stream, s->kp,
                       (const T*)(s->base + s->L.pop[s->cur]), part);
}
template <class T, bool W> static void launch_tips(dlb3_solver* s, int cx, int cy, int cz, double* out) {
    hipLaunchKernelGGL((k3_tips<T, W>), dim3(1), dim3(64), 0, s->stream, s->kp, (const T*)(s->base + s->L.pop[s->cur]),
                       cx, cy, cz, out);
}

#define DISPATCH3(s, fn, ...)                                                     \
    do {                                                                          \
        switch ((s)->p.precision) {                                               \
        case DLB3_F64:                                                            \
            if ((s)->p.walls) fn<double, true>(s, ##__VA_ARGS__);                 \
            else fn<double, false>(s, ##__VA_ARGS__);                             \
            break;                                                                \
        case DLB3_F32:                                                            \
            if ((s)->p.walls) fn<float, true>(s, ##__VA_ARGS__);                  \
            else fn<float, false>(s, ##__VA_ARGS__);                              \
            break;                                                                \
        case DLB3_F16S:                                                           \
            if ((s)->p.walls) fn<__half, true>(s, ##__VA_ARGS__);                 \
            else fn<__half, false>(s, ##__VA_ARGS__);                             \
            break;                                                                \
        default:                                                                  \
            if ((s)->p.walls) fn<__hip_bfloat16, true>(s, ##__VA_ARGS__);         \
            else fn<__hip_bfloat16, false>(s, ##__VA_ARGS__);                     \
        }                                                                         \
    } while (0)

extern "C" {

const char* dlb3_last_error(void) { return g_err3.c_str(); }

size_t dlb3_state_bytes(const dlb3_params* p) {
    if (check3(p) != DLB3_OK) return 0;
    return layout3(p).total;
}

int dlb3_create(const dlb3_params* p, void* dev_state, size_t bytes, void* hip_stream, dlb3_handle* out) {
    int rc = check3(p);
    if (rc) return rc;
    if (!out || !dev_state) return fail3(DLB3_EINVAL, "null state or handle pointer");
    Layout3 L = layout3(p);
    if (bytes < L.total) return fail3(DLB3_ENOMEM, "state buffer smaller than dlb3_state_bytes");
    if (((uintptr_t)dev_state) % 256) return fail3(DLB3_EINVAL, "state buffer must be 256-byte aligned");
    dlb3_solver* s = new (std::nothrow) dlb3_solver();
    if (!s) return fail3(DLB3_ENOMEM, "host allocation failed");
    s->p = *p;
    s->L = L;
    s->kp = make_k3(p, L);
    s->base = (char*)dev_state;
    s->stream = (hipStream_t)hip_stream;
    s->cur = 0;
    s->fcur = 0;
    s->hist_valid = 0;
    s->grid = dim3(s->kp.nb);
    s->block = dim3(BX, BY);
    *out = s;
    return DLB3_OK;
}

int dlb3_destroy(dlb3_handle h) {
    delete h;
    return DLB3_OK;
}

int dlb3_set_fields(dlb3_handle s, const double* phi, const double* C, const double* theta, const double* ux,
                    const double* uy, const double* uz) {
    if (!s || !phi) return fail3(DLB3_EINVAL, "null handle or phi");
    const size_t N = (size_t)s->p.nx * s->p.ny * s->p.nz;
    double* st = (double*)(s->base + s->L.stage);
    const double* srcs[6] = {phi, C, theta, ux, uy, uz};
    for (int j = 0; j < 6; ++j) {
        if (!srcs[j]) continue;
        hipError_t e = hipMemcpyAsync(st + j * s->L.plane, srcs[j], N * sizeof(double), hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return hip_fail3(e, "hipMemcpyAsync");
    }
    const size_t P = s->L.plane;
    DISPATCH3(s, launch_set, st, C ? st + P : nullptr, theta ? st + 2 * P : nullptr, ux ? st + 3 * P : nullptr,
              uy ? st + 4 * P : nullptr, uz ? st + 5 * P : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail3(e, "k3_set");
    // the host arrays must stay valid until the copies ran
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail3(e, "hipStreamSynchronize");
    s->hist_valid = 0;
    return DLB3_OK;
}

int dlb3_init_seed(dlb3_handle s) {
    if (!s) return fail3(DLB3_EINVAL, "null handle");
    double* st = (double*)(s->base + s->L.stage);
    hipLaunchKernelGGL(k3_seed, s->grid, s->block, 0, s->stream, s->kp, s->p.seed_R, s->p.seed_x, s->p.seed_y,
                       s->p.seed_z, s->p.W0, st);
    DISPATCH3(s, launch_set, st, nullptr, nullptr, nullptr, nullptr, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail3(e, "k3_seed/k3_set");
    s->hist_valid = 0;
    return DLB3_OK;
}

int dlb3_step(dlb3_handle s, int64_t n) {
    if (!s || n < 0) return fail3(DLB3_EINVAL, "null handle or negative step count");
    for (int64_t t = 0; t < n; ++t) {
        DISPATCH3(s, launch_step);
        s->cur ^= 1;
        s->hist_valid = 1;
        if (s->p.use_ns)  // sub-steps at the frozen phi of time t (hist plane 0)
            for (int j = 0; j < s->p.n_sub; ++j) {
                DISPATCH3(s, launch_flow);
                s->fcur ^= 1;
            }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail3(e, "k3_step");
    return DLB3_OK;
}

int dlb3_get_fields(dlb3_handle s, double* out) {
    if (!s || !out) return fail3(DLB3_EINVAL, "null handle or output");
    const size_t N = (size_t)s->p.nx * s->p.ny * s->p.nz;
    double* st = (double*)(s->base + s->L.stage);
    DISPATCH3(s, launch_fields, st);
    hipError_t e = hipMemcpyAsync(out, st, 8 * N * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail3(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail3(e, "hipStreamSynchronize");
    return DLB3_OK;
}

int dlb3_reduce(dlb3_handle s, double* out) {
    if (!s || !out) return fail3(DLB3_EINVAL, "null handle or output");
    double* st = (double*)(s->base + s->L.stage);
    const size_t nb = (size_t)s->grid.x * s->grid.y;
    if (4 * nb + 10 > 8 * s->L.plane) return fail3(DLB3_EINVAL, "staging area too small for the reduction");
    double* res = st + 4 * nb;  // 4 sums, then 6 tips
    DISPATCH3(s, launch_partial, st);
    hipLaunchKernelGGL(k3_final, dim3(1), dim3(256), 0, s->stream, (const double*)st, (int)nb, res);
    const int cx = (int)std::lround(s->p.seed_x), cy = (int)std::lround(s->p.seed_y), cz = (int)std::lround(s->p.seed_z);
    DISPATCH3(s, launch_tips, cx, cy, cz, res + 4);
    double host[10];
    hipError_t e = hipMemcpyAsync(host, res, sizeof host, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail3(e, "reduce copy");
    out[0] = host[0];
    out[1] = host[1];
    out[2] = host[2] / ((double)s->p.nx * s->p.ny * s->p.nz);
    out[3] = host[3];
    for (int a = 0; a < 6; ++a) out[4 + a] = host[4 + a];
    return DLB3_OK;
}

}  // extern "C"
