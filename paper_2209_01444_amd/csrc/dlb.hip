// dlb.hip -- host runtime and C ABI of libdlb.so (see include/dlb.h).
//
// The solver binds to a caller-owned device buffer and stream.  A main step
// is one k_pct launch followed by N_sub k_flow launches, all on that stream;
// long runs replay a captured HIP graph of two main steps (two steps bring
// both ping-pong buffers back to the same parity, so one graph serves every
// replay).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "dlb.h"
#include "batch.h"
#include "kernels.h"

#include <algorithm>
#include <vector>

using namespace dlb;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(DLB_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t storage_bytes(int precision) {
    switch (precision) {
        case DLB_F64: return 8;
        case DLB_F32:
        case DLB_F32M: return 4;
        case DLB_F16S:
        case DLB_BF16S:
        case DLB_F16SM: return 2;
    }
    return 0;
}
// history planes are FP64 only in the all-FP64 configuration
size_t history_bytes(int precision) { return precision == DLB_F64 ? 8 : 4; }
// solute and heat populations: FP32 in mixed storage, else the storage type
size_t cde_bytes(int precision) { return precision == DLB_F16SM ? 4 : storage_bytes(precision); }
// byte offset of the five heat planes in a population buffer
size_t heat_offset(int precision, size_t plane) {
    return 5 * plane * storage_bytes(precision) + 5 * plane * cde_bytes(precision);
}

struct Layout {
    size_t plane;  // elements per plane
    size_t pop[2], flow[2], hist, phin, aux, heat, red, redout, total;
    int nblocks;
};

int check_params(const dlb_params* p) {
    if (!p) return fail(DLB_EINVAL, "null params");
    if (p->nx < 16 || p->ny < 16) return fail(DLB_EINVAL, "grid must be at least 16x16");
    if ((long long)p->nx * p->ny > (1ll << 31)) return fail(DLB_EINVAL, "grid too large");
    if (storage_bytes(p->precision) == 0) return fail(DLB_EINVAL, "unknown precision");
    if (p->bc != DLB_BC_PERIODIC && p->bc != DLB_BC_CHANNEL && p->bc != DLB_BC_FARFIELD)
        return fail(DLB_EINVAL, "unknown bc");
    if (p->use_ns && p->n_sub < 1) return fail(DLB_EINVAL, "n_sub must be >= 1");
    if (p->phi_static != 0 && p->phi_static != 1) return fail(DLB_EINVAL, "phi_static must be 0 or 1");
    if (p->isothermal != 0 && p->isothermal != 1) return fail(DLB_EINVAL, "isothermal must be 0 or 1");
    if (p->grad_stencil != 0 && p->grad_stencil != 1) return fail(DLB_EINVAL, "grad_stencil must be 0 or 1");
    if (p->n_sub_t < 0 || p->n_sub_t > 256) return fail(DLB_EINVAL, "n_sub_t must be in [0, 256]");
    if (p->tile_rows != 0 && p->tile_rows != 32 && p->tile_rows != 48)
        return fail(DLB_EINVAL, "tile_rows must be 0 (automatic), 32 or 48");
    const bool forced = p->force_x != 0.0 || p->force_y != 0.0 || p->varphi != 0.0;
    if (!(std::isfinite(p->force_x) && std::isfinite(p->force_y) && std::isfinite(p->varphi)))
        return fail(DLB_EINVAL, "force and varphi must be finite");
    if (forced && !p->use_ns) return fail(DLB_EINVAL, "an external force or varphi needs the flow lattice");
    if (forced && p->flow_fuse > 1)
        return fail(DLB_EUNSUPPORTED, "with an external force or varphi each flow sub-step is one launch (flow_fuse 0 or 1)");
    if (p->bc == DLB_BC_FARFIELD && (p->use_ns || p->grad_stencil || p->n_sub_t > 1 || p->phi_static))
        return fail(DLB_EUNSUPPORTED,
                    "far-field walls need use_ns = 0, grad_stencil = 0, n_sub_t <= 1 and phi_static = 0");
    if (!(p->W0 > 0 && p->tau0 > 0 && p->D > 0 && p->alpha > 0)) return fail(DLB_EINVAL, "W0, tau0, D, alpha must be > 0");
    if (!(p->k > 0 && p->k < 1)) return fail(DLB_EINVAL, "partition coefficient k must be in (0,1)");
    double W2t = p->W0 * p->W0 / p->tau0;
    double lo = 1.0 - p->eps4, hi = 1.0 + p->eps4;  // range of a_s
    const double nt = p->n_sub_t > 1 ? p->n_sub_t : 1;  // heat sub-steps
    double rates[4] = {1.0 / (3.0 * lo * lo * W2t + 0.5), 1.0 / (3.0 * p->D * (1.0 - p->k) + 0.5),
                       1.0 / (3.0 * p->alpha / nt + 0.5), 1.0};
    double r2 = 1.0 / (3.0 * hi * hi * W2t + 0.5);
    if (p->use_ns) {
        if (!(p->nu > 0)) return fail(DLB_EINVAL, "nu must be > 0");
        rates[3] = 1.0 / (3.0 * p->nu / p->n_sub + 0.5);
        // the incompressible D2Q9 model's error grows with Ma^2; the paper's
        // cylinder runs at u = 0.1 per sub-step (Ma = 0.17)
        double mach = std::sqrt(p->u_in_x * p->u_in_x + p->u_in_y * p->u_in_y) / p->n_sub * std::sqrt(3.0);
        if (mach > 0.3) return fail(DLB_EINVAL, "inflow Mach number |u| sqrt(3)/N_sub exceeds 0.3");
    }
    for (double r : rates)
        if (!(r > 0.0 && r < 2.0)) return fail(DLB_EINVAL, "relaxation rate outside (0,2)");
    if (!(r2 > 0.0 && r2 < 2.0)) return fail(DLB_EINVAL, "relaxation rate outside (0,2)");
    if (!(p->eps4 >= 0.0 && p->eps4 < 1.0 / 15.0)) return fail(DLB_EINVAL, "eps4 must be in [0, 1/15)");
    return DLB_OK;
}

Layout layout_of(const dlb_params* p) {
    Layout L{};
    size_t N = (size_t)p->nx * p->ny;
    L.plane = (N + 63) & ~size_t(63);
    size_t sb = storage_bytes(p->precision), cb = history_bytes(p->precision), sc = cde_bytes(p->precision);
    size_t off = 0;
    for (int b = 0; b < 2; ++b) {
        L.pop[b] = off;
        off = align256(off + 5 * L.plane * sb + 10 * L.plane * sc);
    }
    for (int b = 0; b < 2; ++b) {
        L.flow[b] = off;
        if (p->use_ns) off = align256(off + 9 * L.plane * sb);
    }
    L.hist = off;
    off = align256(off + (p->use_ns ? 6 : 2) * L.plane * cb);
    L.phin = off;  // phi at time t for the stencil-gradient ablation
    if (p->grad_stencil) off = align256(off + L.plane * cb);
    const bool heat_split = p->n_sub_t > 1 && !p->isothermal;
    L.aux = off;  // u and d_t(Hu) of time t for the heat sub-steps
    if (heat_split) off = align256(off + 4 * L.plane * cb);
    L.heat = off;  // five heat planes: intermediate heat sub-steps
    if (heat_split) off = align256(off + 5 * L.plane * sc);
    int nbx = (p->nx + TILE_X - 1) / TILE_X, nby = (p->ny + TILE_Y - 1) / TILE_Y;
    L.nblocks = nbx * nby;
    L.red = off;
    off = align256(off + (size_t)L.nblocks * NRED * sizeof(double));
    L.redout = off;
    off = align256(off + 32 * sizeof(double));
    L.total = off;
    return L;
}

}  // namespace

// Rest-state populations used as storage shifts for the 16-bit formats:
// liquid phi = -1, the initial far-field C and theta, inflow velocity.
static void rest_shifts(const dlb_params* p, float* sh) {
    const double w5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
    double phi = -1.0, k = p->k;
    double C = p->c_init_U ? 0.5 * (1.0 + k - (1.0 - k) * phi) * (1.0 + (1.0 - k) * p->U0) : p->C0;
    double U = (2.0 * C / (1.0 + k - (1.0 - k) * phi) - 1.0) / (1.0 - k);
    double ux = p->use_ns ? p->u_in_x : 0.0, uy = p->use_ns ? p->u_in_y : 0.0;
    double q = 0.5 * (1.0 - phi), qU = q * U;
    double H = p->theta0 - 0.5 * phi;  // h(-1) = -1 for both forms of h
    int cx[5] = {0, 1, 0, -1, 0}, cy[5] = {0, 0, 1, 0, -1};
    for (int i = 0; i < 5; ++i) {
        sh[i] = (float)(w5[i] * phi);
        double cu = cx[i] * C * ux + cy[i] * C * uy;
        sh[5 + i] = (float)(i == 0 ? C + (w5[0] - 1.0) * qU : w5[i] * qU + w5[i] * 3.0 * cu);
        double hu = cx[i] * H * ux + cy[i] * H * uy;
        sh[10 + i] = (float)(i == 0 ? w5[0] * p->theta0 - 0.5 * phi : w5[i] * p->theta0 + w5[i] * 3.0 * hu);
    }
    const double w9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    int c9x[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, c9y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    double n = p->use_ns ? p->n_sub : 1;
    double vx = ux / n, vy = uy / n, uu = vx * vx + vy * vy;
    for (int i = 0; i < 9; ++i) {
        double cu = c9x[i] * vx + c9y[i] * vy;
        sh[15 + i] = (float)(w9[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

static KParams make_kparams(const dlb_params* p, const Layout& L) {
    KParams k{};
    k.nx = p->nx;
    k.ny = p->ny;
    k.plane = (long long)L.plane;
    k.n_sub = p->use_ns ? p->n_sub : 1;
    k.h_quintic = p->h_quintic;
    // fixed-point defaults per arithmetic type of the phi/C/theta kernel:
    // FP64 to 1e-14, FP64 arithmetic over FP32 storage (f32m, and f32, whose
    // phi/C/theta kernel computes in FP64) to 1e-10, FP32 to 1e-6
    bool f64 = p->precision == DLB_F64,
         mixed = p->precision == DLB_F32M || p->precision == DLB_F32 || p->precision == DLB_F16SM;
    k.grad_iters = p->grad_iters > 0 ? p->grad_iters : (f64 ? 100 : (mixed ? 40 : 20));
    double tol = p->grad_tol > 0 ? p->grad_tol : (f64 ? 1e-14 : (mixed ? 1e-10 : 1e-6));
    k.grad_tol2 = tol * tol;
    k.walls = p->bc != DLB_BC_PERIODIC;
    k.farfield = p->bc == DLB_BC_FARFIELD;
    // far-field liquid: the initial C at phi = -1 (uniform C0, or that of U0)
    k.ff_C = p->c_init_U ? 1.0 + (1.0 - p->k) * p->U0 : p->C0;
    k.ff_U = (k.ff_C - 1.0) / (1.0 - p->k);
    // external force per flow sub-step and the varphi pressure term
    // 3 varphi K with K = 2 (s2 - 3 s4 + s2 s4) / (9 s2 s4), s4 = 1
    k.force = p->use_ns && (p->force_x != 0.0 || p->force_y != 0.0 || p->varphi != 0.0);
    k.fx_sub = k.force ? p->force_x / ((double)k.n_sub * k.n_sub) : 0.0;
    k.fy_sub = k.force ? p->force_y / ((double)k.n_sub * k.n_sub) : 0.0;
    k.varphi = k.force ? p->varphi : 0.0;
    {
        const double s2 = p->use_ns ? 1.0 / (3.0 * p->nu / p->n_sub + 0.5) : 1.0, s4 = 1.0;
        k.kpf = 3.0 * k.varphi * 2.0 * (s2 - 3.0 * s4 + s2 * s4) / (9.0 * s2 * s4);
    }
    k.use_t = p->isothermal ? 0 : 1;
    k.theta0 = p->theta0;
    k.nbx = (p->nx + TILE_X - 1) / TILE_X;
    k.nby = (p->ny + TILE_Y - 1) / TILE_Y;
    k.nblocks = L.nblocks;
    k.W0 = p->W0;
    k.W2t = p->W0 * p->W0 / p->tau0;
    k.inv_tau0 = 1.0 / p->tau0;
    k.eps4 = p->eps4;
    k.orient = p->orient;
    k.co = std::cos(p->orient);
    k.so = std::sin(p->orient);
    k.lambda = p->lambda;
    k.Mcinf = p->Mcinf;
    k.k = p->k;
    k.invD = 1.0 / p->D;
    k.s1c = 1.0 / (3.0 * p->D * (1.0 - p->k) + 0.5);
    k.n_sub_t = (p->n_sub_t > 1 && !p->isothermal) ? p->n_sub_t : 1;  // k.aux is set with the buffer
    k.s1t = 1.0 / (3.0 * p->alpha / k.n_sub_t + 0.5);
    k.s2u = p->use_ns ? 1.0 / (3.0 * p->nu / p->n_sub + 0.5) : 1.0;
    k.jat = p->W0 / (2.0 * std::sqrt(2.0));
    k.nsub_d = k.n_sub;
    k.uin_x_sub = p->u_in_x / k.n_sub;
    k.uin_y_sub = p->u_in_y / k.n_sub;
    k.seed_R = p->seed_R;
    k.seed_x = p->seed_x;
    k.seed_y = p->seed_y;
    k.noise_amp = p->noise_amp;
    if (p->precision == DLB_F16S || p->precision == DLB_BF16S || p->precision == DLB_F16SM) rest_shifts(p, k.shift);
    for (int t = 0; t < 2; ++t)  // wave-row fused tiles of 8 and 12 waves, K = 3 and 5 (-1: no valid shift)
        for (int j = 0; j < 2; ++j)
            k.tbw_dy[t][j] = tbw_row_shift(p->ny, j ? 5 : 3, k.walls != 0, &k.tbw_nby[t][j],
                                           t ? TbWaveT<TBW_TALL_NW>::EY : TbWave::EY);
    k.tbw_tall = 0;  // chosen in dlb_create
    k.grad_stencil = p->grad_stencil;  // k.phin is set once the state buffer is known
    return k;
}

// ---------------------------------------------------------------------------
// Kernel dispatch per (storage type, flow on, walls)
// ---------------------------------------------------------------------------
struct Ops {
    void (*pct)(const KParams&, const void*, void*, const void*, void*, int, hipStream_t, dim3);
    void (*phi_plane)(const KParams&, const void*, void*, hipStream_t, dim3);
    void (*heat_sub)(const KParams&, const void*, void*, const void*, hipStream_t, dim3);
    void (*flow)(const KParams&, const void*, void*, const void*, hipStream_t, dim3);
    // K fused sub-steps (K in {3, 5}); returns false if K is not built
    bool (*flow_tb)(int, const KParams&, const void*, void*, const void*, hipStream_t);
    void (*set_fields)(const KParams&, const InitFields&, void*, void*, void*, hipStream_t, dim3);
    void (*restart_prep)(const KParams&, const void*, const void*, void*, double*, int, hipStream_t,
                         dim3);
    void (*fields)(const KParams&, const void*, const void*, uint32_t, void*, int, hipStream_t, dim3);
    void (*reduce)(const KParams&, const void*, const void*, double*, hipStream_t, dim3);
    void (*tips)(const KParams&, const void*, double*, hipStream_t);
};

struct BatchOps {
    void (*pct)(char*, const SeedDesc*, int, int, int, int, int, int, hipStream_t);
    void (*flow)(char*, const SeedDesc*, int, int, int, int, int, hipStream_t);
    void (*flow_tb)(int, char*, const SeedDesc*, int, int, int, int, hipStream_t);
};

template <class CF, bool NS, bool W> struct OpsImpl {
    using S = typename CF::S;
    using H = typename CF::H;
    // configuration of the phi/C/theta kernels: same storage, their own arithmetic
    using CP = typename PctArith<CF>::type;
    static void pct(const KParams& kp, const void* pin, void* pout, const void* hin, void* hist,
                    int hv, hipStream_t st, dim3 grid) {
        if constexpr (NS) {
            if (kp.force) {
                hipLaunchKernelGGL((k_pct_force<CP, W>), grid, dim3(BLOCK), 0, st, kp, (const S*)pin, (S*)pout,
                                   (const S*)hin, (H*)hist, hv);
                return;
            }
        }
        hipLaunchKernelGGL((k_pct<CP, NS, W>), grid, dim3(BLOCK), 0, st, kp, (const S*)pin, (S*)pout,
                           (const S*)hin, (H*)hist, hv);
    }
    static void phi_plane(const KParams& kp, const void* pin, void* phin, hipStream_t st, dim3 grid) {
        hipLaunchKernelGGL((k_phi_plane<CP, W>), grid, dim3(BLOCK), 0, st, kp, (const S*)pin, (H*)phin);
    }
    static void heat_sub(const KParams& kp, const void* gin, void* gout, const void* hist, hipStream_t st,
                         dim3 grid) {
        using SC = typename CF::SC;
        hipLaunchKernelGGL((k_heat_sub<CP, W>), grid, dim3(BLOCK), 0, st, kp, (const SC*)gin, (SC*)gout,
                           (const H*)hist);
    }
    static void flow(const KParams& kp, const void* hin, void* hout, const void* phi, hipStream_t st,
                     dim3 grid) {
        if constexpr (NS) {
            if (kp.force) {
                hipLaunchKernelGGL((k_flow_force<CF, W>), grid, dim3(BLOCK), 0, st, kp, (const S*)hin, (S*)hout,
                                   (const H*)phi);
                return;
            }
        }
        hipLaunchKernelGGL((k_flow<CF, W>), grid, dim3(BLOCK), 0, st, kp, (const S*)hin, (S*)hout,
                           (const H*)phi);
    }
    template <int K>
    static void tb_launch(const KParams& kp, const void* hin, void* hout, const void* phi,
                          hipStream_t st) {
        using T = typename CF::T;
        using G = TbGeom<T>;
        constexpr int OX = G::EX - 2 * K, OY = G::EY - 2 * K;
        const int nbx = (kp.nx + OX - 1) / OX;
        const int nby = sizeof(T) == 4 ? kp.tbw_nby[0][K == 5] : (kp.ny + OY - 1) / OY;
        if constexpr (sizeof(T) == 4) {
            if (kp.tbw_tall) {
                constexpr int NWT = TBW_TALL_NW, OYT = TbWaveT<NWT>::EY - 2 * K;
                static_assert(OYT > 0, "tall tile");
                const int nbt = kp.tbw_nby[1][K == 5];
                hipLaunchKernelGGL((k_flow_tbw<CF, W, K, NWT>), dim3(nbx * nbt), dim3(64 * NWT), 0, st, kp,
                                   (const S*)hin, (S*)hout, (const H*)phi, nbx, nbx * nbt);
                return;
            }
            hipLaunchKernelGGL((k_flow_tbw<CF, W, K>), dim3(nbx * nby), dim3(G::THREADS), 0, st, kp,
                               (const S*)hin, (S*)hout, (const H*)phi, nbx, nbx * nby);
        } else
            hipLaunchKernelGGL((k_flow_tb<CF, W, G::EX, G::EY, K>), dim3(nbx * nby), dim3(G::THREADS), 0, st,
                               kp, (const S*)hin, (S*)hout, (const H*)phi, nbx, nbx * nby);
    }
    static bool flow_tb(int K, const KParams& kp, const void* hin, void* hout, const void* phi,
                        hipStream_t st) {
        switch (K) {
            case 3: tb_launch<3>(kp, hin, hout, phi, st); return true;
            case 5: tb_launch<5>(kp, hin, hout, phi, st); return true;
        }
        return false;
    }
    static void set_fields(const KParams& kp, const InitFields& in, void* pop, void* flow, void* hist,
                           hipStream_t st, dim3 grid) {
        hipLaunchKernelGGL((k_set_fields<CP, NS, W>), grid, dim3(BLOCK), 0, st, kp, in, (S*)pop,
                           (S*)flow, (H*)hist);
    }
    static void restart_prep(const KParams& kp, const void* pop, const void* flow, void* hist,
                             double* phi_old, int hv, hipStream_t st, dim3 grid) {
        hipLaunchKernelGGL((k_restart_prep<CP, NS, W>), grid, dim3(BLOCK), 0, st, kp, (const S*)pop,
                           (const S*)flow, (H*)hist, phi_old, hv);
    }
    static void fields(const KParams& kp, const void* pop, const void* flow, uint32_t mask, void* out,
                       int f32, hipStream_t st, dim3 grid) {
        hipLaunchKernelGGL((k_fields<CP, NS, W>), grid, dim3(BLOCK), 0, st, kp, (const S*)pop,
                           (const S*)flow, mask, out, f32);
    }
    static void reduce(const KParams& kp, const void* pop, const void* flow, double* partial,
                       hipStream_t st, dim3 grid) {
        hipLaunchKernelGGL((k_reduce_partial<CP, NS, W>), grid, dim3(BLOCK), 0, st, kp,
                           (const S*)pop, (const S*)flow, partial);
    }
    static void tips(const KParams& kp, const void* pop, double* out, hipStream_t st) {
        hipLaunchKernelGGL((k_tips<CP, W>), dim3(4), dim3(448), 0, st, kp, (const S*)pop, out);
    }
    static Ops ops() {
        return Ops{pct, phi_plane, heat_sub, flow, flow_tb, set_fields, restart_prep, fields, reduce, tips};
    }

    // batched persistent launches
    static void b_pct(char* base, const SeedDesc* d, int count, int total, int cur, int fcur, int tw_log2,
                      int blocks, hipStream_t st) {
        hipLaunchKernelGGL((k_pct_batch<CP, NS, W>), dim3(blocks), dim3(BLOCK), 0, st, base, d, count, total,
                           cur, fcur, tw_log2);
    }
    static void b_flow(char* base, const SeedDesc* d, int count, int total, int fcur, int tw_log2, int blocks,
                       hipStream_t st) {
        hipLaunchKernelGGL((k_flow_batch<CF, W>), dim3(blocks), dim3(BLOCK), 0, st, base, d, count, total,
                           fcur, tw_log2);
    }
    static void b_flow_tb(int K, char* base, const SeedDesc* d, int count, int total, int fcur, int blocks,
                          hipStream_t st) {
        constexpr int TH = TbGeom<typename CF::T>::THREADS;
        if (K == 3)
            hipLaunchKernelGGL((k_flow_tb_batch<CF, W, 3>), dim3(blocks), dim3(TH), 0, st, base, d, count,
                               total, fcur);
        else
            hipLaunchKernelGGL((k_flow_tb_batch<CF, W, 5>), dim3(blocks), dim3(TH), 0, st, base, d, count,
                               total, fcur);
    }
    static BatchOps bops() { return BatchOps{b_pct, b_flow, b_flow_tb}; }
};

template <class CF> static Ops ops_for(bool ns, bool walls) {
    if (ns) return walls ? OpsImpl<CF, true, true>::ops() : OpsImpl<CF, true, false>::ops();
    return walls ? OpsImpl<CF, false, true>::ops() : OpsImpl<CF, false, false>::ops();
}

template <class CF> static BatchOps bops_for(bool ns, bool walls) {
    if (ns) return walls ? OpsImpl<CF, true, true>::bops() : OpsImpl<CF, true, false>::bops();
    return walls ? OpsImpl<CF, false, true>::bops() : OpsImpl<CF, false, false>::bops();
}

static BatchOps select_bops(const dlb_params* p) {
    bool ns = p->use_ns != 0, walls = p->bc != DLB_BC_PERIODIC;
    switch (p->precision) {
        case DLB_F64: return bops_for<CfgF64>(ns, walls);
        case DLB_F32: return bops_for<CfgF32>(ns, walls);
        case DLB_F32M: return bops_for<CfgF32M>(ns, walls);
        case DLB_F16S: return bops_for<CfgF16>(ns, walls);
        case DLB_F16SM: return bops_for<CfgF16M>(ns, walls);
        default: return bops_for<CfgBF16>(ns, walls);
    }
}

static Ops select_ops(const dlb_params* p) {
    bool ns = p->use_ns != 0, walls = p->bc != DLB_BC_PERIODIC;
    switch (p->precision) {
        case DLB_F64: return ops_for<CfgF64>(ns, walls);
        case DLB_F32: return ops_for<CfgF32>(ns, walls);
        case DLB_F32M: return ops_for<CfgF32M>(ns, walls);
        case DLB_F16S: return ops_for<CfgF16>(ns, walls);
        case DLB_F16SM: return ops_for<CfgF16M>(ns, walls);
        default: return ops_for<CfgBF16>(ns, walls);
    }
}

struct dlb_solver {
    dlb_params p;
    Layout L;
    KParams kp;
    Ops ops;
    char* base;
    size_t bytes;
    hipStream_t stream;
    int pop_cur = 0, flow_cur = 0;
    int hist_valid = 0;
    int64_t step = 0;
    dim3 grid;
    int fuse = 1;                    // flow sub-steps fused per launch
    int batched = 0;                 // member of a batch: stepped by the batch only
    hipGraphExec_t graph = nullptr;  // two main steps, valid once history is valid
    int graph_pop = -1, graph_flow = -1;

    void* pop(int b) const { return base + L.pop[b]; }
    void* flow(int b) const { return base + L.flow[b]; }
    void* hist() const { return base + L.hist; }
    double* red() const { return (double*)(base + L.red); }
    double* redout() const { return (double*)(base + L.redout); }
};

// Enqueue one main step.  Events, when given (3 of them), are recorded
// before the phi/C/theta kernel, between it and the flow sub-steps, and after
// the last sub-step, so the N_sub flow kernels run back to back as in a plain
// step.
static void enqueue_step(dlb_solver* s, hipEvent_t* ev) {
    if (ev) (void)hipEventRecord(ev[0], s->stream);
    if (!s->p.phi_static) {
        if (s->p.grad_stencil) s->ops.phi_plane(s->kp, s->pop(s->pop_cur), s->base + s->L.phin, s->stream, s->grid);
        s->ops.pct(s->kp, s->pop(s->pop_cur), s->pop(1 - s->pop_cur), s->flow(s->flow_cur), s->hist(),
                   s->hist_valid, s->stream, s->grid);
        if (s->kp.n_sub_t > 1) {
            // heat sub-steps from the current buffer's heat planes to the new
            // buffer's, alternating with the scratch planes so the last one
            // lands in the new buffer
            const size_t off = heat_offset(s->p.precision, s->L.plane);
            char* from = (char*)s->pop(s->pop_cur) + off;
            char* dst = (char*)s->pop(1 - s->pop_cur) + off;
            char* scr = s->base + s->L.heat;
            const int nt = s->kp.n_sub_t;
            for (int j = 0; j < nt; ++j) {
                char* to = ((nt - 1 - j) % 2 == 0) ? dst : scr;
                s->ops.heat_sub(s->kp, from, to, s->hist(), s->stream, s->grid);
                from = to;
            }
        }
        s->pop_cur ^= 1;
        s->hist_valid = 1;
    }
    if (ev) (void)hipEventRecord(ev[1], s->stream);
    if (s->p.use_ns) {
        // K fused sub-steps per launch while K fit, single sub-steps after
        int left = s->p.n_sub;
        const int K = s->fuse;
        while (K > 1 && left >= K) {
            s->ops.flow_tb(K, s->kp, s->flow(s->flow_cur), s->flow(1 - s->flow_cur), s->hist(),
                           s->stream);
            s->flow_cur ^= 1;
            left -= K;
        }
        for (; left > 0; --left) {
            s->ops.flow(s->kp, s->flow(s->flow_cur), s->flow(1 - s->flow_cur), s->hist(), s->stream,
                        s->grid);
            s->flow_cur ^= 1;
        }
    }
    if (ev) (void)hipEventRecord(ev[2], s->stream);
    s->step += 1;
}

static int build_graph(dlb_solver* s) {
    if (s->graph) {
        (void)hipGraphExecDestroy(s->graph);
        s->graph = nullptr;
    }
    hipGraph_t g;
    int pc = s->pop_cur, fc = s->flow_cur;
    int64_t st = s->step;
    HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    enqueue_step(s, nullptr);
    enqueue_step(s, nullptr);
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    s->pop_cur = pc;
    s->flow_cur = fc;
    s->step = st;
    if (e != hipSuccess) return fail(DLB_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        s->graph = nullptr;
        return fail(DLB_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    s->graph_pop = pc;
    s->graph_flow = fc;
    return DLB_OK;
}

extern "C" {

const char* dlb_last_error(void) { return g_last_error.c_str(); }

const char* dlb_strerror(int code) {
    switch (code) {
        case DLB_OK: return "ok";
        case DLB_EINVAL: return "invalid argument";
        case DLB_ENOMEM: return "state buffer too small";
        case DLB_EHIP: return "HIP error";
        case DLB_ENAN: return "non-finite values detected";
        case DLB_EUNSUPPORTED: return "unsupported combination";
    }
    return "unknown error";
}

size_t dlb_state_bytes(const dlb_params* p) {
    if (check_params(p) != DLB_OK) return 0;
    return layout_of(p).total;
}

int dlb_create(const dlb_params* p, void* dev_state, size_t bytes, void* hip_stream, dlb_handle* out) {
    if (!out) return fail(DLB_EINVAL, "null output handle");
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    Layout L = layout_of(p);
    if (!dev_state || bytes < L.total)
        return fail(DLB_ENOMEM, "state buffer smaller than dlb_state_bytes()");
    if (((uintptr_t)dev_state & 255) != 0) return fail(DLB_EINVAL, "state buffer must be 256-byte aligned");
    dlb_solver* s = new (std::nothrow) dlb_solver();
    if (!s) return fail(DLB_ENOMEM, "host allocation failed");
    s->p = *p;
    s->L = L;
    s->kp = make_kparams(p, L);
    if (s->kp.tbw_dy[0][0] < 0 || s->kp.tbw_dy[0][1] < 0) {  // not reached for ny >= 3
        delete s;
        return fail(DLB_EUNSUPPORTED, "no row shift of the fused flow tiles fits this grid height");
    }
    s->ops = select_ops(p);
    s->base = (char*)dev_state;
    s->kp.phin = p->grad_stencil ? s->base + L.phin : nullptr;
    s->kp.aux = s->kp.n_sub_t > 1 ? s->base + L.aux : nullptr;
    s->bytes = bytes;
    s->stream = (hipStream_t)hip_stream;
    s->grid = dim3(L.nblocks);
    // default fuse depth: 5 for the wave-row tile (FP32 flow arithmetic), 3
    // for the LDS tile of FP64 flow arithmetic, whose 64-bit tile at K = 5
    // keeps too few workgroups resident (f64 3,940 against 3,550 MLUPS at
    // 1024^2, f32m 5,650 against 4,430)
    const bool fp64_flow = p->precision == DLB_F64 || p->precision == DLB_F32M;
    s->fuse = p->flow_fuse == 0 ? (s->kp.force ? 1 : (fp64_flow ? 3 : 5)) : p->flow_fuse;
    if (s->fuse != 1 && s->fuse != 3 && s->fuse != 5) {
        delete s;
        return fail(DLB_EINVAL, "flow_fuse must be 0 (default), 1, 3 or 5");
    }
    // fused tile height (FP32 flow arithmetic): 48 rows on grids whose tall
    // tiles fill at least four rounds of the resident slots (two tiles per
    // compute unit), where the smaller halo pays; 32 rows otherwise, where the
    // launch's last round would run few tiles
    const bool tall_ok = !fp64_flow && s->fuse > 1 && s->kp.tbw_dy[1][s->fuse == 5] >= 0;
    if (p->tile_rows == 48 && !tall_ok) {
        delete s;
        return fail(DLB_EUNSUPPORTED, "tile_rows 48 needs FP32 flow arithmetic, fused sub-steps and a row shift "
                                      "that fits the grid");
    }
    if (p->tile_rows == 0 && tall_ok) {
        int dev = 0, ncu = 256;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
            ncu = 256;
        const int OX = TbWave::EX - 2 * s->fuse;
        const long tiles = (long)((p->nx + OX - 1) / OX) * s->kp.tbw_nby[1][s->fuse == 5];
        s->kp.tbw_tall = tiles >= 4L * 2 * ncu;
    } else {
        s->kp.tbw_tall = p->tile_rows == 48;
    }
    *out = s;
    return DLB_OK;
}

int dlb_destroy(dlb_handle h) {
    if (!h) return fail(DLB_EINVAL, "null handle");
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    delete h;
    return DLB_OK;
}

static int set_fields_device(dlb_handle h, const double* phi, const double* C, const double* th,
                             const double* ux, const double* uy, unsigned flags = 0u) {
    const bool keep_neq = (flags & DLB_KEEP_NONEQ) != 0;
    // phi of the current state goes to the idle ping-pong population buffer
    // (at least 15 planes of 2-byte values per node, room for one double),
    // which the next step overwrites
    double* phi_old = keep_neq ? (double*)h->pop(1 - h->pop_cur) : nullptr;
    int hv = keep_neq ? h->hist_valid : 0;
    if (keep_neq)
        h->ops.restart_prep(h->kp, h->pop(h->pop_cur), h->flow(h->flow_cur), h->hist(), phi_old, hv,
                            h->stream, h->grid);
    InitFields in{phi, C, th, ux, uy, h->p.C0, h->p.U0, h->p.theta0, h->p.u_in_x, h->p.u_in_y,
                  h->p.c_init_U, h->p.use_ns, flags, hv, phi_old, h->p.phi_static};
    h->ops.set_fields(h->kp, in, h->pop(h->pop_cur), h->flow(h->flow_cur), h->hist(), h->stream,
                      h->grid);
    HIP_TRY(hipGetLastError());
    h->hist_valid = hv;
    return DLB_OK;
}

int dlb_set_fields(dlb_handle h, const double* phi, const double* C, const double* theta,
                   const double* ux, const double* uy, int on_device) {
    return dlb_set_fields_ex(h, phi, C, theta, ux, uy, on_device, 0u);
}

int dlb_set_fields_ex(dlb_handle h, const double* phi, const double* C, const double* theta,
                      const double* ux, const double* uy, int on_device, uint32_t flags) {
    if (!h || !phi) return fail(DLB_EINVAL, "null handle or phi");
    if (flags & ~(uint32_t)(DLB_KEEP_FLOW | DLB_KEEP_NONEQ)) return fail(DLB_EINVAL, "unknown flag");
    if (on_device) return set_fields_device(h, phi, C, theta, ux, uy, flags);
    size_t N = (size_t)h->p.nx * h->p.ny;
    const double* src[5] = {phi, C, theta, ux, uy};
    double* tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, 5 * N * sizeof(double)));
    const double* dev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = DLB_OK;
    for (int i = 0; i < 5 && rc == DLB_OK; ++i) {
        if (!src[i]) continue;
        hipError_t e = hipMemcpyAsync(tmp + i * N, src[i], N * sizeof(double), hipMemcpyHostToDevice,
                                      h->stream);
        if (e != hipSuccess) rc = fail(DLB_EHIP, hipGetErrorString(e));
        dev[i] = tmp + i * N;
    }
    if (rc == DLB_OK) rc = set_fields_device(h, dev[0], dev[1], dev[2], dev[3], dev[4], flags);
    hipError_t e = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (rc == DLB_OK && e != hipSuccess) rc = fail(DLB_EHIP, hipGetErrorString(e));
    return rc;
}

int dlb_init_seed(dlb_handle h, const double* noise) {
    if (!h) return fail(DLB_EINVAL, "null handle");
    size_t N = (size_t)h->p.nx * h->p.ny;
    double* tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, 2 * N * sizeof(double)));
    int rc = DLB_OK;
    double* dnoise = nullptr;
    if (noise) {
        hipError_t e = hipMemcpyAsync(tmp + N, noise, N * sizeof(double), hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) rc = fail(DLB_EHIP, hipGetErrorString(e));
        dnoise = tmp + N;
    }
    if (rc == DLB_OK) {
        hipLaunchKernelGGL(k_seed_phi, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, h->stream, h->kp,
                           (const double*)dnoise, tmp);
        rc = set_fields_device(h, tmp, nullptr, nullptr, nullptr, nullptr);
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (rc == DLB_OK && e != hipSuccess) rc = fail(DLB_EHIP, hipGetErrorString(e));
    return rc;
}

int dlb_step(dlb_handle h, int64_t n) {
    if (!h || n < 0) return fail(DLB_EINVAL, "null handle or negative step count");
    if (h->batched) return fail(DLB_EINVAL, "a batch member is stepped by dlb_batch_step only");
    int64_t done = 0;
    // the first step after (re-)initialisation runs with zero time derivatives
    while (done < n && !h->hist_valid) {
        enqueue_step(h, nullptr);
        ++done;
    }
    // graphs need a capturable (non-null) stream
    if (n - done >= 4 && h->stream != nullptr) {
        if (!h->graph || h->graph_pop != h->pop_cur || h->graph_flow != h->flow_cur) {
            int rc = build_graph(h);
            if (rc) return rc;
        }
        while (n - done >= 2) {
            HIP_TRY(hipGraphLaunch(h->graph, h->stream));
            done += 2;
            h->step += 2;
        }
    }
    while (done < n) {
        enqueue_step(h, nullptr);
        ++done;
    }
    HIP_TRY(hipGetLastError());
    return DLB_OK;
}

int dlb_step_timed(dlb_handle h, int64_t n, double* ms_pct, double* ms_flow, int64_t* l_pct,
                   int64_t* l_flow) {
    if (!h || n < 0) return fail(DLB_EINVAL, "null handle or negative step count");
    if (h->batched) return fail(DLB_EINVAL, "a batch member is stepped by dlb_batch_step only");
    hipEvent_t ev[3];
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    double a = 0.0, b = 0.0;
    int64_t la = 0, lb = 0;
    int rc = DLB_OK;
    for (int64_t s = 0; s < n && rc == DLB_OK; ++s) {
        enqueue_step(h, ev);
        hipError_t e = hipEventSynchronize(ev[2]);
        if (e != hipSuccess) {
            rc = fail(DLB_EHIP, hipGetErrorString(e));
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
        a += ms;
        ++la;
        if (h->p.use_ns) {
            (void)hipEventElapsedTime(&ms, ev[1], ev[2]);
            b += ms;
            lb += h->p.n_sub / h->fuse + h->p.n_sub % h->fuse;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (ms_pct) *ms_pct = a;
    if (ms_flow) *ms_flow = b;
    if (l_pct) *l_pct = la;
    if (l_flow) *l_flow = lb;
    return rc;
}

int64_t dlb_step_count(dlb_handle h) { return h ? h->step : -1; }

int dlb_get_fields(dlb_handle h, uint32_t mask, void* out, int out_on_device, int out_f32) {
    if (!h || !out) return fail(DLB_EINVAL, "null handle or output");
    if (mask == 0 || mask >= (1u << 7)) return fail(DLB_EINVAL, "field mask must select bits 0..6");
    size_t N = (size_t)h->p.nx * h->p.ny;
    int nf = __builtin_popcount(mask);
    size_t bytes = (size_t)nf * N * (out_f32 ? 4 : 8);
    void* dst = out;
    if (!out_on_device) HIP_TRY(hipMalloc(&dst, bytes));
    h->ops.fields(h->kp, h->pop(h->pop_cur), h->flow(h->flow_cur), mask, dst, out_f32, h->stream,
                  h->grid);
    hipError_t e = hipGetLastError();
    if (!out_on_device) {
        if (e == hipSuccess) e = hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        (void)hipFree(dst);
    }
    if (e != hipSuccess) return fail(DLB_EHIP, hipGetErrorString(e));
    return DLB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Static staging buffer of dlb_get_fields_noalloc: a file-scope device array
// (each GPU holds its own copy for the life of the process).  Host code never
// passes the array's name to a kernel or a copy: the name is a host-side
// stand-in, so its device address is looked up once per device and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[DLB_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`; looked up with that
// device current on the first call for it.
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(DLB_EUNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return fail(DLB_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DLB_OK;
}
}  // namespace

extern "C" {

int dlb_get_fields_noalloc(dlb_handle h, uint32_t mask, void* out, int out_f32) {
    if (!h || !out) return fail(DLB_EINVAL, "null handle or output");
    if (mask == 0 || mask >= (1u << 7)) return fail(DLB_EINVAL, "field mask must select bits 0..6");
    const size_t N = (size_t)h->p.nx * h->p.ny;
    const size_t bytes = (size_t)__builtin_popcount(mask) * N * (out_f32 ? 4 : 8);
    if (bytes > (size_t)DLB_NOALLOC_SCRATCH_BYTES)
        return fail(DLB_EINVAL, "selected fields exceed the static staging buffer (DLB_NOALLOC_SCRATCH_BYTES)");
    hipPointerAttribute_t attr;
    HIP_TRY(hipPointerGetAttributes(&attr, h->base));
    void* scr = nullptr;
    int rc = scratch_address(attr.device, &scr);
    if (rc) return rc;
    // k_fields writes every selected value, so nothing needs clearing first
    h->ops.fields(h->kp, h->pop(h->pop_cur), h->flow(h->flow_cur), mask, scr, out_f32, h->stream, h->grid);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, scr, bytes, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return DLB_OK;
}

int dlb_reduce(dlb_handle h, double* out) {
    if (!h || !out) return fail(DLB_EINVAL, "null handle or output");
    h->ops.reduce(h->kp, h->pop(h->pop_cur), h->flow(h->flow_cur), h->red(), h->stream, h->grid);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(BLOCK), 0, h->stream, (const double*)h->red(),
                       h->L.nblocks, (long long)h->p.nx * h->p.ny, h->redout());
    h->ops.tips(h->kp, h->pop(h->pop_cur), h->redout(), h->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, h->redout(), 19 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (out[3] > 0) return fail(DLB_ENAN, "non-finite values in the state");
    return DLB_OK;
}

static const uint64_t CKPT_MAGIC = 0x444c42434b505431ull;  // "DLBCKPT1"
struct CkptHeader {
    uint64_t magic;
    dlb_params p;
    int64_t step;
    int32_t pop_cur, flow_cur, hist_valid, pad;
    uint64_t state_bytes;
};

size_t dlb_checkpoint_bytes(dlb_handle h) { return h ? sizeof(CkptHeader) + h->L.total : 0; }

int dlb_save(dlb_handle h, void* host, size_t bytes) {
    if (!h || !host) return fail(DLB_EINVAL, "null handle or buffer");
    if (bytes < dlb_checkpoint_bytes(h)) return fail(DLB_ENOMEM, "checkpoint buffer too small");
    CkptHeader hd{CKPT_MAGIC, h->p, h->step, h->pop_cur, h->flow_cur, h->hist_valid, 0, h->L.total};
    std::memcpy(host, &hd, sizeof hd);
    HIP_TRY(hipMemcpyAsync((char*)host + sizeof hd, h->base, h->L.total, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return DLB_OK;
}

int dlb_load(dlb_handle h, const void* host, size_t bytes) {
    if (!h || !host) return fail(DLB_EINVAL, "null handle or buffer");
    if (h->batched) return fail(DLB_EINVAL, "a batch member cannot load a checkpoint");
    if (bytes < sizeof(CkptHeader)) return fail(DLB_EINVAL, "checkpoint truncated");
    CkptHeader hd;
    std::memcpy(&hd, host, sizeof hd);
    if (hd.magic != CKPT_MAGIC) return fail(DLB_EINVAL, "not a checkpoint");
    if (std::memcmp(&hd.p, &h->p, sizeof(dlb_params)) != 0)
        return fail(DLB_EINVAL, "checkpoint parameters differ from the solver's");
    if (hd.state_bytes != h->L.total || bytes < sizeof hd + hd.state_bytes)
        return fail(DLB_EINVAL, "checkpoint size mismatch");
    HIP_TRY(hipMemcpyAsync(h->base, (const char*)host + sizeof hd, h->L.total, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->step = hd.step;
    h->pop_cur = hd.pop_cur;
    h->flow_cur = hd.flow_cur;
    h->hist_valid = hd.hist_valid;
    return DLB_OK;
}

int dlb_copy_state(dlb_handle dst, dlb_handle src) {
    if (!dst || !src) return fail(DLB_EINVAL, "null handle");
    if (std::memcmp(&dst->p, &src->p, sizeof(dlb_params)) != 0)
        return fail(DLB_EINVAL, "solvers have different parameters");
    if (dst->batched) return fail(DLB_EINVAL, "cannot overwrite a batch member");
    HIP_TRY(hipMemcpyAsync(dst->base, src->base, src->L.total, hipMemcpyDeviceToDevice, src->stream));
    if (dst->stream != src->stream) HIP_TRY(hipStreamSynchronize(src->stream));
    dst->step = src->step;
    dst->pop_cur = src->pop_cur;
    dst->flow_cur = src->flow_cur;
    dst->hist_valid = src->hist_valid;
    return DLB_OK;
}

int dlb_sync(dlb_handle h) {
    if (!h) return fail(DLB_EINVAL, "null handle");
    HIP_TRY(hipStreamSynchronize(h->stream));
    return DLB_OK;
}

int dlb_equilibria(int64_t n, const double* macros, double* out, int h_quintic) {
    if (n <= 0 || !macros || !out) return fail(DLB_EINVAL, "bad arguments");
    double *din = nullptr, *dout = nullptr;
    HIP_TRY(hipMalloc(&din, (size_t)n * 8 * sizeof(double)));
    hipError_t e = hipMalloc(&dout, (size_t)n * 24 * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(din, macros, (size_t)n * 8 * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_equilibria, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, (long long)n,
                           (const double*)din, dout, h_quintic);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, (size_t)n * 24 * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(din);
    if (dout) (void)hipFree(dout);
    if (e != hipSuccess) return fail(DLB_EHIP, hipGetErrorString(e));
    return DLB_OK;
}

int dlb_copy_kernel(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
        return fail(DLB_EINVAL, "copy needs 16-byte aligned pointers and size");
    size_t n = bytes / 16;
    unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 256 * 16);
    if (blocks == 0) return DLB_OK;
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4*)src,
                       (float4*)dst, n);
    HIP_TRY(hipGetLastError());
    return DLB_OK;
}


// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
}  // extern "C"

struct dlb_batch {
    int count = 0;
    dlb_params p0;  // shared precision / flow / walls / n_sub
    std::vector<dlb_solver*> members;
    std::vector<SeedDesc> desc;
    SeedDesc* d_desc = nullptr;
    char* base = nullptr;  // the caller's state buffer: member arrays are offsets into it
    int total_tiles = 0, total_tb[2] = {0, 0};
    hipStream_t stream = nullptr;
    int pop_cur = 0, flow_cur = 0;
    int64_t step = 0;
    int fuse = 5, bpc_node = 4096, bpc_tb = 4096, num_cu = 256;  // grids: one tile per workgroup
    int node_tw_log2 = 6;  // node tiles of 64 x 4 nodes
    BatchOps ops;
    hipGraphExec_t graph = nullptr;
    int graph_pop = -1, graph_flow = -1;
};

extern "C" int dlb_batch_destroy(dlb_batch_handle b);

static bool batch_compatible(const dlb_params* a, const dlb_params* b) {
    return a->precision == b->precision && a->use_ns == b->use_ns && a->bc == b->bc &&
           (!a->use_ns || a->n_sub == b->n_sub);
}

static int batch_layout(const dlb_params* ps, int count, std::vector<size_t>* offs, size_t* total) {
    if (!ps || count < 1) return fail(DLB_EINVAL, "empty batch");
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        int rc = check_params(&ps[i]);
        if (rc) return rc;
        if (ps[i].phi_static) return fail(DLB_EUNSUPPORTED, "phi_static is not available in batches");
        if (ps[i].bc == DLB_BC_FARFIELD) return fail(DLB_EUNSUPPORTED, "far-field walls are not available in batches");
        if (ps[i].force_x != 0.0 || ps[i].force_y != 0.0 || ps[i].varphi != 0.0)
            return fail(DLB_EUNSUPPORTED, "an external force or varphi is not available in batches");
        if (ps[i].grad_stencil) return fail(DLB_EUNSUPPORTED, "grad_stencil is not available in batches");
        if (ps[i].n_sub_t > 1) return fail(DLB_EUNSUPPORTED, "n_sub_t > 1 is not available in batches");
        if (!batch_compatible(&ps[0], &ps[i]))
            return fail(DLB_EINVAL, "batch members must share precision, use_ns, bc and n_sub");
        if (offs) offs->push_back(off);
        off = align256(off + layout_of(&ps[i]).total);
    }
    off = align256(off + (size_t)count * sizeof(SeedDesc));
    *total = off;
    return DLB_OK;
}

static int upload_desc(dlb_batch* b) {
    for (int i = 0; i < b->count; ++i) {
        dlb_solver* m = b->members[i];
        b->desc[i].hist_valid = m->hist_valid;
    }
    HIP_TRY(hipMemcpyAsync(b->d_desc, b->desc.data(), b->desc.size() * sizeof(SeedDesc),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return DLB_OK;
}

// Node-kernel work list for tiles of 2^tw_log2 x (BLOCK >> tw_log2) nodes:
// each member's first tile and tiles per row; the caller uploads it.
static void batch_node_tiles(dlb_batch* b, int tw_log2) {
    const int tw = 1 << tw_log2, th = BLOCK >> tw_log2;
    b->total_tiles = 0;
    for (int i = 0; i < b->count; ++i) {
        const dlb_params& p = b->members[i]->p;
        const int nbx = (p.nx + tw - 1) / tw, nby = (p.ny + th - 1) / th;
        b->desc[i].tile0 = b->total_tiles;
        b->desc[i].node_nbx = nbx;
        b->total_tiles += nbx * nby;
    }
    b->node_tw_log2 = tw_log2;
}

// Batch grids are a multiple of the 8 XCDs, so that batch_span gives every
// XCD one contiguous band of the work list (a grid trimmed to the item count
// would otherwise interleave the items over the XCDs); surplus workgroups
// find their range empty.
static int batch_grid(int items, int num_cu, int per_cu) { return (std::min(items, num_cu * per_cu) + 7) & ~7; }

static void batch_enqueue_step(dlb_batch* b, int fuse, int bpc_node, int bpc_tb) {
    const int bn = batch_grid(b->total_tiles, b->num_cu, bpc_node);
    b->ops.pct(b->base, b->d_desc, b->count, b->total_tiles, b->pop_cur, b->flow_cur, b->node_tw_log2, bn,
               b->stream);
    b->pop_cur ^= 1;
    if (b->p0.use_ns) {
        int left = b->p0.n_sub;
        while (fuse > 1 && left >= fuse) {
            int L = fuse == 5 ? 1 : 0;
            const int bt = batch_grid(b->total_tb[L], b->num_cu, bpc_tb);
            b->ops.flow_tb(fuse, b->base, b->d_desc, b->count, b->total_tb[L], b->flow_cur, bt, b->stream);
            b->flow_cur ^= 1;
            left -= fuse;
        }
        for (; left > 0; --left) {
            b->ops.flow(b->base, b->d_desc, b->count, b->total_tiles, b->flow_cur, b->node_tw_log2, bn,
                        b->stream);
            b->flow_cur ^= 1;
        }
    }
    b->step += 1;
}

static void batch_sync_members(dlb_batch* b) {
    for (dlb_solver* m : b->members) {
        m->pop_cur = b->pop_cur;
        m->flow_cur = b->flow_cur;
        m->step = b->step;
        m->hist_valid = 1;
    }
}

extern "C" {

size_t dlb_batch_state_bytes(const dlb_params* ps, int count) {
    size_t total = 0;
    if (batch_layout(ps, count, nullptr, &total) != DLB_OK) return 0;
    return total;
}

int dlb_batch_create(const dlb_params* ps, int count, void* dev_state, size_t bytes, void* hip_stream,
                     dlb_batch_handle* out) {
    if (!out) return fail(DLB_EINVAL, "null output handle");
    *out = nullptr;
    std::vector<size_t> offs;
    size_t total = 0;
    int rc = batch_layout(ps, count, &offs, &total);
    if (rc) return rc;
    if (!dev_state || bytes < total) return fail(DLB_ENOMEM, "state buffer smaller than dlb_batch_state_bytes()");
    if (((uintptr_t)dev_state & 255) != 0) return fail(DLB_EINVAL, "state buffer must be 256-byte aligned");
    dlb_batch* b = new (std::nothrow) dlb_batch();
    if (!b) return fail(DLB_ENOMEM, "host allocation failed");
    b->count = count;
    b->p0 = ps[0];
    b->stream = (hipStream_t)hip_stream;
    b->base = (char*)dev_state;
    b->ops = select_bops(&ps[0]);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        b->num_cu = ncu;
    const bool f64 = ps[0].precision == DLB_F64 || ps[0].precision == DLB_F32M;
    const int EX = f64 ? TbGeom<double>::EX : TbGeom<float>::EX;
    const int EY = f64 ? TbGeom<double>::EY : TbGeom<float>::EY;
    for (int i = 0; i < count; ++i) {
        dlb_handle m = nullptr;
        rc = dlb_create(&ps[i], (char*)dev_state + offs[i], layout_of(&ps[i]).total, hip_stream, &m);
        if (rc) {
            for (dlb_solver* x : b->members) dlb_destroy(x);
            delete b;
            return rc;
        }
        m->batched = 1;
        b->members.push_back(m);
        SeedDesc d{};
        d.kp = m->kp;
        d.pop[0] = (size_t)((char*)m->pop(0) - b->base);
        d.pop[1] = (size_t)((char*)m->pop(1) - b->base);
        d.flow[0] = (size_t)((char*)m->flow(0) - b->base);
        d.flow[1] = (size_t)((char*)m->flow(1) - b->base);
        d.hist = (size_t)((char*)m->hist() - b->base);
        const int Ks[2] = {3, 5};
        for (int L = 0; L < 2; ++L) {
            int OX = EX - 2 * Ks[L], OY = EY - 2 * Ks[L];
            int nbx = (ps[i].nx + OX - 1) / OX, nby = f64 ? (ps[i].ny + OY - 1) / OY : m->kp.tbw_nby[0][L];
            d.tb0[L] = b->total_tb[L];
            d.tb_nbx[L] = nbx;
            b->total_tb[L] += nbx * nby;
        }
        b->desc.push_back(d);
    }
    batch_node_tiles(b, 6);
    b->d_desc = (SeedDesc*)((char*)dev_state + total - align256((size_t)count * sizeof(SeedDesc)));
    rc = upload_desc(b);
    if (rc) {
        dlb_batch_destroy(b);
        return rc;
    }
    *out = b;
    return DLB_OK;
}

int dlb_batch_destroy(dlb_batch_handle b) {
    if (!b) return fail(DLB_EINVAL, "null batch");
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (dlb_solver* m : b->members) dlb_destroy(m);
    delete b;
    return DLB_OK;
}

dlb_handle dlb_batch_member(dlb_batch_handle b, int i) {
    if (!b || i < 0 || i >= b->count) {
        fail(DLB_EINVAL, "member index out of range");
        return nullptr;
    }
    return b->members[i];
}

int dlb_batch_set_config(dlb_batch_handle b, int fuse, int bpc_node, int bpc_tb) {
    if (!b) return fail(DLB_EINVAL, "null batch");
    if ((fuse != 1 && fuse != 3 && fuse != 5) || bpc_node < 1 || bpc_node > 4096 || bpc_tb < 1 || bpc_tb > 4096)
        return fail(DLB_EINVAL, "fuse in {1,3,5}, workgroups per CU in [1,4096] (node and fused)");
    b->fuse = fuse;
    b->bpc_node = bpc_node;
    b->bpc_tb = bpc_tb;
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return DLB_OK;
}

int dlb_batch_set_node_tile(dlb_batch_handle b, int tile_width) {
    if (!b) return fail(DLB_EINVAL, "null batch");
    int lg = -1;
    for (int k = 5; k <= 8; ++k)
        if (tile_width == (1 << k)) lg = k;
    if (lg < 0) return fail(DLB_EINVAL, "node tile width must be 32, 64, 128 or 256");
    batch_node_tiles(b, lg);
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return upload_desc(b);
}

int dlb_batch_get_node_tile(dlb_batch_handle b) {
    if (!b) return fail(DLB_EINVAL, "null batch");
    return 1 << b->node_tw_log2;
}

int dlb_batch_get_config(dlb_batch_handle b, int* out3) {
    if (!b || !out3) return fail(DLB_EINVAL, "null argument");
    out3[0] = b->fuse;
    out3[1] = b->bpc_node;
    out3[2] = b->bpc_tb;
    return DLB_OK;
}

int dlb_batch_step(dlb_batch_handle b, int64_t n) {
    if (!b || n < 0) return fail(DLB_EINVAL, "null batch or negative step count");
    if (n == 0) return DLB_OK;
    bool any_invalid = false, changed = false;
    for (int i = 0; i < b->count; ++i) {
        any_invalid |= !b->members[i]->hist_valid;
        changed |= b->desc[i].hist_valid != b->members[i]->hist_valid;
    }
    if (changed) {
        int rc = upload_desc(b);
        if (rc) return rc;
    }
    int64_t done = 0;
    if (any_invalid) {  // one step with zero time derivatives where re-initialised
        batch_enqueue_step(b, b->fuse, b->bpc_node, b->bpc_tb);
        batch_sync_members(b);
        ++done;
        int rc = upload_desc(b);
        if (rc) return rc;
    }
    if (n - done >= 4 && b->stream != nullptr) {
        if (!b->graph || b->graph_pop != b->pop_cur || b->graph_flow != b->flow_cur) {
            if (b->graph) (void)hipGraphExecDestroy(b->graph);
            b->graph = nullptr;
            int pc = b->pop_cur, fc = b->flow_cur;
            int64_t st = b->step;
            hipGraph_t g;
            HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            batch_enqueue_step(b, b->fuse, b->bpc_node, b->bpc_tb);
            batch_enqueue_step(b, b->fuse, b->bpc_node, b->bpc_tb);
            hipError_t e = hipStreamEndCapture(b->stream, &g);
            b->pop_cur = pc;
            b->flow_cur = fc;
            b->step = st;
            if (e != hipSuccess) return fail(DLB_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                b->graph = nullptr;
                return fail(DLB_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
            }
            b->graph_pop = pc;
            b->graph_flow = fc;
        }
        while (n - done >= 2) {
            HIP_TRY(hipGraphLaunch(b->graph, b->stream));
            done += 2;
            b->step += 2;
        }
    }
    while (done < n) {
        batch_enqueue_step(b, b->fuse, b->bpc_node, b->bpc_tb);
        ++done;
    }
    HIP_TRY(hipGetLastError());
    batch_sync_members(b);
    return DLB_OK;
}

// Time `steps` batch steps of one launch configuration with HIP events.
static int batch_time(dlb_batch* b, int fuse, int bn, int bt, int steps, float* ms) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    batch_enqueue_step(b, fuse, bn, bt);  // warm-up
    (void)hipEventRecord(e0, b->stream);
    for (int i = 0; i < steps; ++i) batch_enqueue_step(b, fuse, bn, bt);
    (void)hipEventRecord(e1, b->stream);
    hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(DLB_EHIP, hipGetErrorString(e));
    return DLB_OK;
}

int dlb_batch_autotune(dlb_batch_handle b, int trial_steps, double* ms_best) {
    if (!b || trial_steps < 1) return fail(DLB_EINVAL, "null batch or trial_steps < 1");
    int rc = upload_desc(b);
    if (rc) return rc;
    const int fuses[3] = {5, 3, 1}, bns[6] = {4, 16, 64, 256, 1024, 4096}, bts[6] = {1, 2, 3, 4, 32, 4096};
    float best = 1e30f;
    int bf = b->fuse, bn = b->bpc_node, bt = b->bpc_tb;
    // coordinate search: fused-launch shape first, then the node-kernel grid
    for (int f : fuses) {
        if (b->p0.use_ns && f > b->p0.n_sub) continue;
        for (int t : bts) {
            if (f == 1 && t != bts[0]) continue;
            float ms = 0.f;
            rc = batch_time(b, f, bn, t, trial_steps, &ms);
            if (rc) return rc;
            if (ms < best) best = ms, bf = f, bt = t;
        }
    }
    for (int n : bns) {
        float ms = 0.f;
        rc = batch_time(b, bf, n, bt, trial_steps, &ms);
        if (rc) return rc;
        if (ms < best) best = ms, bn = n;
    }
    // node tile shape among 64 x 4, 128 x 2, 256 x 1 and 32 x 8; the one the
    // batch holds now was timed above
    const int cur = b->node_tw_log2;
    int blg = cur;
    for (int lg : {6, 7, 8, 5}) {
        if (lg == cur) continue;
        batch_node_tiles(b, lg);
        rc = upload_desc(b);
        if (rc) return rc;
        float ms = 0.f;
        rc = batch_time(b, bf, bn, bt, trial_steps, &ms);
        if (rc) return rc;
        if (ms < best) best = ms, blg = lg;
    }
    rc = dlb_batch_set_node_tile(b, 1 << blg);
    if (rc) return rc;
    rc = dlb_batch_set_config(b, bf, bn, bt);
    if (rc) return rc;
    // the trial steps consumed the state: members must be (re-)initialised
    b->step = 0;
    for (dlb_solver* m : b->members) {
        m->hist_valid = 0;
        m->step = 0;
        m->pop_cur = b->pop_cur;
        m->flow_cur = b->flow_cur;
    }
    if (ms_best) *ms_best = best / trial_steps;
    return DLB_OK;
}

int64_t dlb_batch_step_count(dlb_batch_handle b) { return b ? b->step : -1; }

}  // extern "C"
