// sur.hip -- learned surrogate for gfx950: U-Net forward, backward and Adam
// with bfloat16 matrix-core (MFMA) convolutions.  C ABI in include/sur.h.
//
// Layout: activations NHWC bf16 with channel counts that are multiples of
// 32; 3x3 weights [ky][kx][Cout][Cin] (Cin contiguous).  A 3x3 convolution is
// an implicit GEMM: rows = pixels, columns = output channels, depth = 9 x Cin.
// v_mfma_f32_16x16x32_bf16 lane layout (checked by sur_mfma_check): lane l
// holds A[l%16][8(l/16) .. 8(l/16)+7], B[8(l/16) .. +7][l%16], and returns
// D[4(l/16) + r][l%16], r = 0..3.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "sur.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float LEAK = 0.1f;

thread_local std::string g_err;
int fail(int code, const std::string& m) {
    g_err = m;
    return code;
}
#define HIP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(-3, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

__device__ __forceinline__ float bf2f(bf16 v) { return (float)v; }
__device__ __forceinline__ bf16 f2bf(float v) { return (bf16)v; }

// ---------------------------------------------------------------------------
// 3x3 convolution, forward (also used for the input gradient with flipped,
// transposed weights).  Workgroup: a tile of 4 rows x 64 pixels of one image
// and 16 NJ output channels; wave w computes row w as 4 blocks of 16 pixels
// x NJ blocks of 16 channels (4 NJ accumulators).  Per chunk of 32 input
// channels the tile with its one-pixel halo and the chunk's weights for the
// workgroup's channels (all 9 shifts) are staged in LDS (rows padded to 40
// bf16 = 80 B, so the 16 rows a matrix-core operand reads fall in distinct
// banks); the 9 shifts then read both operands from LDS.
// ---------------------------------------------------------------------------
constexpr int CT_X = 64, CT_Y = 4, CT_PAD = 40;
template <int NJ, bool ACT, bool BIAS>
__global__ __launch_bounds__(256) void k_conv3x3(const bf16* __restrict__ X, const bf16* __restrict__ Wt,
                                                 const float* __restrict__ bias, bf16* __restrict__ Y,
                                                 int N, int H, int W, int Cin, int Cout, int ntx, int nty) {
    __shared__ __attribute__((aligned(16))) bf16 sIn[CT_Y + 2][CT_X + 2][CT_PAD];
    __shared__ __attribute__((aligned(16))) bf16 sW[9][16 * NJ][CT_PAD];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = lane & 15, kq = lane >> 4;
    int t = blockIdx.x;
    const int tx = t % ntx;
    t /= ntx;
    const int ty = t % nty, n = t / nty;
    const int x0 = tx * CT_X, y0 = ty * CT_Y;
    const int co0 = blockIdx.y * 16 * NJ;
    f32x4 acc[4][NJ];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[bb][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // chunk staging, software-pipelined: the global loads of chunk c + 1 are
    // issued right after chunk c reaches LDS, so they are in flight while
    // the matrix cores work on chunk c
    constexpr int NI = ((CT_Y + 2) * (CT_X + 2) * 4 + 255) / 256, NWL = (9 * 16 * NJ * 4 + 255) / 256;
    bf16x8 vin[NI], vw[NWL];
    auto load_chunk = [&](int ci) {
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int i = threadIdx.x + 256 * k;
            const int g = i & 3, pix = i >> 2;
            const int yy = pix / (CT_X + 2), xx = pix % (CT_X + 2);
            const int gy = y0 + yy - 1, gx = x0 + xx - 1;
            vin[k] = bf16x8{};
            if (i < (CT_Y + 2) * (CT_X + 2) * 4 && gy >= 0 && gy < H && gx >= 0 && gx < W)
                vin[k] = *(const bf16x8*)(X + (((size_t)n * H + gy) * W + gx) * Cin + ci + 8 * g);
        }
#pragma unroll
        for (int k = 0; k < NWL; ++k) {
            const int i = threadIdx.x + 256 * k;
            const int g = i & 3, q = i >> 2;
            const int co = q % (16 * NJ), sft = q / (16 * NJ);
            if (i < 9 * 16 * NJ * 4)
                vw[k] = *(const bf16x8*)(Wt + ((size_t)sft * Cout + co0 + co) * Cin + ci + 8 * g);
        }
    };
    load_chunk(0);
    for (int ci = 0; ci < Cin; ci += 32) {
        __syncthreads();  // the previous chunk's operands have been read
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int i = threadIdx.x + 256 * k;
            const int g = i & 3, pix = i >> 2;
            if (i < (CT_Y + 2) * (CT_X + 2) * 4)
                *(bf16x8*)&sIn[pix / (CT_X + 2)][pix % (CT_X + 2)][8 * g] = vin[k];
        }
#pragma unroll
        for (int k = 0; k < NWL; ++k) {
            const int i = threadIdx.x + 256 * k;
            const int g = i & 3, q = i >> 2;
            if (i < 9 * 16 * NJ * 4) *(bf16x8*)&sW[q / (16 * NJ)][q % (16 * NJ)][8 * g] = vw[k];
        }
        __syncthreads();
        if (ci + 32 < Cin) load_chunk(ci + 32);
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                bf16x8 bv[NJ];
#pragma unroll
                for (int j = 0; j < NJ; ++j) bv[j] = *(const bf16x8*)&sW[ky * 3 + kx][16 * j + row][8 * kq];
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) {
                    const bf16x8 av = *(const bf16x8*)&sIn[wave + ky][16 * bb + row + kx][8 * kq];
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        acc[bb][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[bb][j], 0, 0, 0);
                }
            }
        }
    }
    const int y = y0 + wave;
    if (y >= H) return;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int co = co0 + j * 16 + row;
        const float bval = BIAS ? bias[co] : 0.f;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int px = x0 + 16 * bb + 4 * kq + r;
                if (px < W) {
                    float v = acc[bb][j][r] + bval;
                    if (ACT) v = v > 0.f ? v : LEAK * v;
                    Y[(((size_t)n * H + y) * W + px) * Cout + co] = f2bf(v);
                }
            }
    }
}

template <int NJ, bool ACT, bool BIAS>
void launch_conv_t(hipStream_t st, const bf16* in, const bf16* wt, const float* bias, bf16* out, int B, int H, int W,
                   int Cin, int Cout) {
    const int ntx = (W + CT_X - 1) / CT_X, nty = (H + CT_Y - 1) / CT_Y;
    dim3 grid((unsigned)(ntx * nty * B), (unsigned)(Cout / (16 * NJ)));
    hipLaunchKernelGGL((k_conv3x3<NJ, ACT, BIAS>), grid, dim3(256), 0, st, in, wt, bias, out, B, H, W, Cin, Cout,
                       ntx, nty);
}

// Y = conv(X, Wt) (+ bias, leaky ReLU); Cin and Cout multiples of 32
void launch_conv(hipStream_t st, const bf16* in, const bf16* wt, const float* bias, bf16* out, int B, int H, int W,
                 int Cin, int Cout, bool act) {
    // 64 output channels per workgroup, unless that leaves fewer than 512
    // workgroups (deep levels at small batch): then 32, for twice as many
    const long long tiles = (long long)((W + CT_X - 1) / CT_X) * ((H + CT_Y - 1) / CT_Y) * B;
    const bool wide = Cout % 64 == 0 && tiles * (Cout / 64) >= 512;
    if (bias) {
        if (wide) {
            if (act) launch_conv_t<4, true, true>(st, in, wt, bias, out, B, H, W, Cin, Cout);
            else launch_conv_t<4, false, true>(st, in, wt, bias, out, B, H, W, Cin, Cout);
        } else {
            if (act) launch_conv_t<2, true, true>(st, in, wt, bias, out, B, H, W, Cin, Cout);
            else launch_conv_t<2, false, true>(st, in, wt, bias, out, B, H, W, Cin, Cout);
        }
    } else {
        if (wide) launch_conv_t<4, false, false>(st, in, wt, nullptr, out, B, H, W, Cin, Cout);
        else launch_conv_t<2, false, false>(st, in, wt, nullptr, out, B, H, W, Cin, Cout);
    }
}

// ---------------------------------------------------------------------------
// 3x3 convolution, weight gradient:  dW[s][co][ci] += sum_m dP[m][co] X_s[m][ci]
// (X_s = X shifted by s, zero outside).  A k-step is a segment of 32
// pixels of one image row; the segment's dP (transposed, [co][px]) and the
// three input rows around it, stored once per column shift kx (transposed,
// [s][ci][px]), are staged in LDS, so one dP operand serves all 9 shifts.
// Workgroup: a CO_T x CI_T (co, ci) tile, all 9 shifts, a run of k-steps;
// wave w owns a fixed set of 16 x 16 blocks and accumulates them in
// registers, then adds them to dW with FP32 atomics.
// ---------------------------------------------------------------------------
constexpr int WG_PX = 32;
template <int CO_T, int CI_T>
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const bf16* __restrict__ X, const bf16* __restrict__ dP,
                                                       float* __restrict__ dW, int N, int H, int W, int Cin,
                                                       int Cout, int nseg, int per_wg) {
    constexpr int NCO = CO_T / 16, NCI = CI_T / 16;
    // wave w: ci block w % NCI, co blocks w / NCI + k (4 / NCI) .. (all 9 shifts)
    constexpr int WCI = NCI >= 4 ? NCI / 4 : 1;           // ci blocks per wave
    constexpr int WCO = NCI >= 4 ? NCO : NCO * NCI / 4;   // co blocks per wave
    constexpr int NACC = 9 * WCO * WCI;
    __shared__ __attribute__((aligned(16))) bf16 sA[CO_T][WG_PX + 8];
    __shared__ __attribute__((aligned(16))) bf16 sX[9][CI_T][WG_PX + 8];
    const int nci_t = Cin / CI_T;
    const int co0 = (blockIdx.y / nci_t) * CO_T, ci0 = (blockIdx.y % nci_t) * CI_T;
    const long long total = (long long)N * H * nseg;
    const long long kbeg = (long long)blockIdx.x * per_wg;
    const long long kend = kbeg + per_wg < total ? kbeg + per_wg : total;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int row = lane & 15, kq = lane >> 4;
    // this wave's blocks
    int cb_first, cb_step, ib_first;
    if (NCI >= 4) {
        ib_first = wave * WCI;
        cb_first = 0;
        cb_step = 1;
    } else {  // NCI in {1, 2}: 4 / NCI waves share the ci blocks, co blocks interleaved
        ib_first = wave % NCI;
        cb_first = wave / NCI;
        cb_step = 4 / NCI;
    }
    f32x4 acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    // k-step staging, software-pipelined: the global loads of step ks + 1
    // are issued once step ks is in LDS, in flight during its products
    constexpr int NA = (WG_PX * (CO_T / 8) + 255) / 256, NX = (3 * (WG_PX + 2) * (CI_T / 8) + 255) / 256;
    bf16x8 va[NA], vx[NX];
    auto load_step = [&](long long ks) {
        const int seg = (int)(ks % nseg);
        const long long ny = ks / nseg;
        const int y = (int)(ny % H), n = (int)(ny / H);
        const int xs = seg * WG_PX;
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int v = tid + 256 * k;
            const int g = v % (CO_T / 8), px = v / (CO_T / 8);
            const int x = xs + px;
            va[k] = bf16x8{};
            if (v < WG_PX * (CO_T / 8) && x < W)
                va[k] = *(const bf16x8*)(dP + (((size_t)n * H + y) * W + x) * Cout + co0 + 8 * g);
        }
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            const int v = tid + 256 * k;
            const int g = v % (CI_T / 8), q = v / (CI_T / 8);
            const int xx = q % (WG_PX + 2), ky = q / (WG_PX + 2);
            const int gy = y + ky - 1, gx = xs + xx - 1;
            vx[k] = bf16x8{};
            if (v < 3 * (WG_PX + 2) * (CI_T / 8) && gy >= 0 && gy < H && gx >= 0 && gx < W)
                vx[k] = *(const bf16x8*)(X + (((size_t)n * H + gy) * W + gx) * Cin + ci0 + 8 * g);
        }
    };
    if (kbeg < kend) load_step(kbeg);
    for (long long ks = kbeg; ks < kend; ++ks) {
        __syncthreads();  // the previous step's operands have been read
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int v = tid + 256 * k;
            const int g = v % (CO_T / 8), px = v / (CO_T / 8);
            if (v < WG_PX * (CO_T / 8))
#pragma unroll
                for (int e = 0; e < 8; ++e) sA[8 * g + e][px] = va[k][e];
        }
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            const int v = tid + 256 * k;
            const int g = v % (CI_T / 8), q = v / (CI_T / 8);
            const int xx = q % (WG_PX + 2), ky = q / (WG_PX + 2);
            if (v < 3 * (WG_PX + 2) * (CI_T / 8)) {
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const int px = xx - kx;  // pixel xs + px takes input column xs + px + kx - 1
                    if (px >= 0 && px < WG_PX) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) sX[ky * 3 + kx][8 * g + e][px] = vx[k][e];
                    }
                }
            }
        }
        __syncthreads();
        if (ks + 1 < kend) load_step(ks + 1);
#pragma unroll
        for (int c = 0; c < WCO; ++c) {
            const int cb = cb_first + c * cb_step;
            const bf16x8 av = *(const bf16x8*)&sA[cb * 16 + row][8 * kq];
#pragma unroll
            for (int i = 0; i < WCI; ++i) {
                const int ib = ib_first + i;
#pragma unroll
                for (int sft = 0; sft < 9; ++sft) {
                    const bf16x8 bv = *(const bf16x8*)&sX[sft][ib * 16 + row][8 * kq];
                    f32x4& ac = acc[(c * WCI + i) * 9 + sft];
                    ac = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, ac, 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < WCO; ++c) {
        const int cb = cb_first + c * cb_step;
#pragma unroll
        for (int i = 0; i < WCI; ++i) {
            const int ci = ci0 + (ib_first + i) * 16 + row;
#pragma unroll
            for (int sft = 0; sft < 9; ++sft)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int co = co0 + cb * 16 + 4 * kq + r;
                    atomicAdd(&dW[((size_t)sft * Cout + co) * Cin + ci], acc[(c * WCI + i) * 9 + sft][r]);
                }
        }
    }
}

void launch_wgrad(hipStream_t st, const bf16* X, const bf16* dP, float* dW, int N, int H, int W, int Cin,
                  int Cout, int num_cu) {
    const int nseg = (W + WG_PX - 1) / WG_PX;
    const long long total = (long long)N * H * nseg;
    const bool big = Cin % 64 == 0 && Cout % 64 == 0;
    const int tiles = big ? (Cout / 64) * (Cin / 64) : (Cout / 32) * (Cin / 32);
    // about two workgroups per compute unit in all, at least 8 k-steps each
    long long want = (2ll * num_cu + tiles - 1) / tiles;
    long long per = (total + want - 1) / want;
    if (per < 8) per = 8;
    const unsigned nwg = (unsigned)((total + per - 1) / per);
    dim3 grid(nwg, (unsigned)tiles);
    if (big)
        hipLaunchKernelGGL((k_conv3x3_wgrad<64, 64>), grid, dim3(256), 0, st, X, dP, dW, N, H, W, Cin, Cout, nseg,
                           (int)per);
    else
        hipLaunchKernelGGL((k_conv3x3_wgrad<32, 32>), grid, dim3(256), 0, st, X, dP, dW, N, H, W, Cin, Cout, nseg,
                           (int)per);
}

// bias gradient: db[c] += sum_m dP[m][c].  Thread: 8 channels (one vector)
// of every (256 / (C / 8))-th pixel of the block's pixel range; the block
// reduces through LDS and adds C values with atomics.
__global__ __launch_bounds__(256) void k_bias_grad(const bf16* __restrict__ dP, float* __restrict__ db, long long M,
                                                   int C) {
    __shared__ float red[256][9];
    const int G = C / 8, lanes = 256 / G;  // C in {32, 64, 128, 256}
    const int g = threadIdx.x % G, sub = threadIdx.x / G;
    const long long per = (M + gridDim.x - 1) / gridDim.x;
    const long long beg = blockIdx.x * per, end = beg + per < M ? beg + per : M;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long long m = beg + sub; m < end; m += lanes) {
        const bf16x8 v = *(const bf16x8*)(dP + m * C + 8 * g);
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[e] += bf2f(v[e]);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[threadIdx.x][e] = acc[e];
    __syncthreads();
    if (threadIdx.x < C) {
        const int gg = threadIdx.x / 8, e = threadIdx.x % 8;
        float s = 0.f;
        for (int k = 0; k < lanes; ++k) s += red[k * G + gg][e];
        atomicAdd(&db[threadIdx.x], s);
    }
}

// leaky ReLU backward from the stored output: dY *= (Y > 0 ? 1 : LEAK), 8 per thread
__global__ void k_leaky_bwd(const bf16* __restrict__ Y, bf16* __restrict__ dY, long long n8) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const bf16x8 y = ((const bf16x8*)Y)[i];
    bf16x8 d = ((bf16x8*)dY)[i];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float g = bf2f(d[e]);
        d[e] = f2bf(bf2f(y[e]) > 0.f ? g : LEAK * g);
    }
    ((bf16x8*)dY)[i] = d;
}

// 2x2 average pooling and its adjoint; thread: one pixel, 8 channels
__global__ void k_pool2(const bf16* __restrict__ X, bf16* __restrict__ Y, int N, int H, int W, int C) {
    const int Ho = H / 2, Wo = W / 2, G = C / 8;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)N * Ho * Wo * G) return;
    const int g = (int)(i % G);
    const int p = (int)(i / G);
    const int xo = p % Wo, yo = (p / Wo) % Ho, n = p / (Wo * Ho);
    const size_t b = (((size_t)n * H + 2 * yo) * W + 2 * xo) * C + 8 * g;
    const bf16x8 a0 = *(const bf16x8*)(X + b), a1 = *(const bf16x8*)(X + b + C);
    const bf16x8 a2 = *(const bf16x8*)(X + b + (size_t)W * C), a3 = *(const bf16x8*)(X + b + (size_t)W * C + C);
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = f2bf(0.25f * (bf2f(a0[e]) + bf2f(a1[e]) + bf2f(a2[e]) + bf2f(a3[e])));
    *(bf16x8*)(Y + (size_t)p * C + 8 * g) = o;
}
// dX (full resolution) = dY / 4 broadcast; `accumulate` adds to dX
__global__ void k_pool2_bwd(const bf16* __restrict__ dY, bf16* __restrict__ dX, int N, int H, int W, int C,
                            int accumulate) {
    const int G = C / 8;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)N * H * W * G) return;
    const int g = (int)(i % G);
    const int p = (int)(i / G);
    const int x = p % W, y = (p / W) % H, n = p / (W * H);
    const bf16x8 d = *(const bf16x8*)(dY + (((size_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + 8 * g);
    bf16* out = dX + (size_t)p * C + 8 * g;
    bf16x8 o = accumulate ? *(const bf16x8*)out : bf16x8{};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float gv = 0.25f * bf2f(d[e]);
        o[e] = f2bf(accumulate ? bf2f(o[e]) + gv : gv);
    }
    *(bf16x8*)out = o;
}

// up2(A) concatenated with S along channels: out[.., 0:Ca] = A(y/2, x/2),
// out[.., Ca:] = S; thread: one pixel, 8 channels
__global__ void k_up2_concat(const bf16* __restrict__ A, const bf16* __restrict__ S, bf16* __restrict__ O, int N,
                             int H, int W, int Ca, int Cs) {
    const int C = Ca + Cs, G = C / 8;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)N * H * W * G) return;
    const int c = 8 * (int)(i % G);
    const int p = (int)(i / G);
    const int x = p % W, y = (p / W) % H, n = p / (W * H);
    const bf16x8 v = c < Ca ? *(const bf16x8*)(A + (((size_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * Ca + c)
                            : *(const bf16x8*)(S + (size_t)p * Cs + (c - Ca));
    *(bf16x8*)(O + (size_t)p * C + c) = v;
}
// adjoint: dA (low res) = sum of the four children's first Ca channels; dS = the rest
__global__ void k_up2_concat_bwd(const bf16* __restrict__ dO, bf16* __restrict__ dA, bf16* __restrict__ dS,
                                 int N, int H, int W, int Ca, int Cs) {
    const int C = Ca + Cs, Ho = H / 2, Wo = W / 2, GA = Ca / 8, GS = Cs / 8;
    const long long nA = (long long)N * Ho * Wo * GA, nS = (long long)N * H * W * GS;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nA) {
        const int c = 8 * (int)(i % GA);
        const int p = (int)(i / GA);
        const int xo = p % Wo, yo = (p / Wo) % Ho, n = p / (Wo * Ho);
        const size_t b = (((size_t)n * H + 2 * yo) * W + 2 * xo) * C + c;
        const bf16x8 a0 = *(const bf16x8*)(dO + b), a1 = *(const bf16x8*)(dO + b + C);
        const bf16x8 a2 = *(const bf16x8*)(dO + b + (size_t)W * C), a3 = *(const bf16x8*)(dO + b + (size_t)W * C + C);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = f2bf(bf2f(a0[e]) + bf2f(a1[e]) + bf2f(a2[e]) + bf2f(a3[e]));
        *(bf16x8*)(dA + (size_t)p * Ca + c) = o;
    } else if (i < nA + nS) {
        const long long k = i - nA;
        const int c = 8 * (int)(k % GS);
        const int p = (int)(k / GS);
        *(bf16x8*)(dS + (size_t)p * Cs + c) = *(const bf16x8*)(dO + (size_t)p * C + Ca + c);
    }
}

// weights for the input gradient: Wf[s][ci][co] = W[8 - s][co][ci]
__global__ void k_flip(const bf16* __restrict__ Wt, bf16* __restrict__ Wf, int Cin, int Cout) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9ll * Cin * Cout) return;
    const int co = (int)(i % Cout);
    long long r = i / Cout;
    const int ci = (int)(r % Cin), s = (int)(r / Cin);
    Wf[i] = Wt[((size_t)(8 - s) * Cout + co) * Cin + ci];
}

// input packing: planar FP32 fields -> normalised NHWC bf16 with 32 channels
// (channels 5..31 zero); thread: one pixel
__global__ void k_pack(const float* __restrict__ F, bf16* __restrict__ X, int N, int H, int W, float m0, float m1,
                       float m2, float m3, float m4, float s0, float s1, float s2, float s3, float s4) {
    const long long hw = (long long)H * W;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (long long)N * hw) return;
    const int n = (int)(p / hw);
    const long long q = p % hw;
    const float mean[5] = {m0, m1, m2, m3, m4}, inv[5] = {1.f / s0, 1.f / s1, 1.f / s2, 1.f / s3, 1.f / s4};
    bf16x8 v = {};
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = f2bf((F[((size_t)n * 5 + c) * hw + q] - mean[c]) * inv[c]);
    bf16x8* out = (bf16x8*)(X + p * 32);
    out[0] = v;
    out[1] = bf16x8{};
    out[2] = bf16x8{};
    out[3] = bf16x8{};
}

// 1x1 head, loss and their gradients.  pred[m][o] = bh[o] + sum_c A[m][c] Wh[o][c];
// with a target T (planar FP32 fields K steps later) and the inputs F:
// r = (T - F)/rstd, loss += sum w_o (pred - r)^2 / count, dpred = 2 w_o (pred - r)/count,
// dA[m][c] = sum_o dpred[o] Wh[o][c].  Without a target, writes F + rstd pred
// as FP64 fields (if out != NULL).
struct HeadArgs {
    float rstd[5];
    float lw[5];  // per-channel loss weights
    float inv_count;
};
__global__ __launch_bounds__(256) void k_head(const bf16* __restrict__ A, const float* __restrict__ Wh,
                                              const float* __restrict__ bh, const float* __restrict__ F,
                                              const float* __restrict__ T, float* __restrict__ dpred,
                                              bf16* __restrict__ dA, double* __restrict__ out,
                                              float* __restrict__ loss, float* __restrict__ dbh, int N, int H, int W,
                                              HeadArgs ha) {
    __shared__ float red[6][4];
    const long long M = (long long)N * H * W;
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long hw = (long long)H * W;
    float lsum = 0.f, dpo[5] = {0, 0, 0, 0, 0};
    if (m < M) {
        float a[32];
        const bf16x8* ap = (const bf16x8*)(A + m * 32);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bf16x8 v = ap[q];
#pragma unroll
            for (int e = 0; e < 8; ++e) a[q * 8 + e] = bf2f(v[e]);
        }
        const int n = (int)(m / hw);
        const long long q = m % hw;
        float pred[5];
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            float s = bh[o];
#pragma unroll
            for (int c = 0; c < 32; ++c) s += a[c] * Wh[o * 32 + c];
            pred[o] = s;
        }
        if (T) {
#pragma unroll
            for (int o = 0; o < 5; ++o) {
                const size_t fi = ((size_t)n * 5 + o) * hw + q;
                float r = (T[fi] - F[fi]) / ha.rstd[o];
                float d = pred[o] - r;
                lsum += ha.lw[o] * d * d * ha.inv_count;
                dpo[o] = 2.f * ha.lw[o] * d * ha.inv_count;
                dpred[m * 5 + o] = dpo[o];
            }
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                float s = 0.f;
#pragma unroll
                for (int o = 0; o < 5; ++o) s += dpo[o] * Wh[o * 32 + c];
                dA[m * 32 + c] = f2bf(s);
            }
        } else if (out) {
#pragma unroll
            for (int o = 0; o < 5; ++o) {
                const size_t fi = ((size_t)n * 5 + o) * hw + q;
                out[fi] = (double)F[fi] + (double)ha.rstd[o] * (double)pred[o];
            }
        }
    }
    if (!T) return;
    float v[6] = {lsum, dpo[0], dpo[1], dpo[2], dpo[3], dpo[4]};
#pragma unroll
    for (int k = 0; k < 6; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int k = 0; k < 6; ++k) red[k][wave] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        float s = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        atomicAdd(threadIdx.x == 0 ? loss : &dbh[threadIdx.x - 1], s);
    }
}
// head weight gradient: dWh[o][c] += sum_m dpred[m][o] A[m][c].  Thread:
// channels 8g..8g+7 of every 64th pixel of the block's range (g = t % 4);
// the block reduces its 160 sums through LDS and adds them with atomics.
__global__ __launch_bounds__(256) void k_head_wgrad(const bf16* __restrict__ A, const float* __restrict__ dpred,
                                                    float* __restrict__ dWh, long long M) {
    __shared__ float red[64][161];
    const int g = threadIdx.x & 3, sub = threadIdx.x >> 2;
    const long long per = (M + gridDim.x - 1) / gridDim.x;
    const long long beg = blockIdx.x * per, end = beg + per < M ? beg + per : M;
    float acc[5][8];
#pragma unroll
    for (int o = 0; o < 5; ++o)
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[o][e] = 0.f;
    for (long long m = beg + sub; m < end; m += 64) {
        const bf16x8 a = *(const bf16x8*)(A + m * 32 + 8 * g);
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            const float d = dpred[m * 5 + o];
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[o][e] += d * bf2f(a[e]);
        }
    }
    // fold the four channel groups of a pixel lane into one row of 160
    for (int gg = 0; gg < 4; ++gg) {
        if (g == gg)
#pragma unroll
            for (int o = 0; o < 5; ++o)
#pragma unroll
                for (int e = 0; e < 8; ++e) red[sub][o * 32 + 8 * gg + e] = acc[o][e];
    }
    __syncthreads();
    if (threadIdx.x < 160) {
        float s = 0.f;
        for (int k = 0; k < 64; ++k) s += red[k][threadIdx.x];
        atomicAdd(&dWh[threadIdx.x], s);
    }
}

__global__ void k_fill(float* __restrict__ p, long long n, float v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_to_bf16(const float* __restrict__ p, bf16* __restrict__ q, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = f2bf(p[i]);
}
// Adam (Kingma and Ba) with bias correction on FP32 master weights
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, bf16* __restrict__ q, long long n, float lr, float c1, float c2) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float gi = g[i];
    float a = b1 * m1[i] + (1.f - b1) * gi;
    float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    float v = p[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    p[i] = v;
    q[i] = f2bf(v);
}

__global__ void k_mfma_check(const bf16* __restrict__ A, const bf16* __restrict__ B, float* __restrict__ D) {
    const int l = threadIdx.x, row = l & 15, kq = l >> 4;
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = A[row * 32 + kq * 8 + e];
        b[e] = B[(kq * 8 + e) * 16 + row];
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) D[(4 * kq + r) * 16 + row] = acc[r];
}

// ---------------------------------------------------------------------------
// Network description
// ---------------------------------------------------------------------------
struct Layer {
    int cin, cin_p, cout, level;  // level: resolution H >> level
    size_t w_off, b_off;          // offsets into the parameter arrays (elements)
};

constexpr int NCONV = 14;
const int LEVEL_CH[4] = {32, 64, 128, 256};

void build_layers(Layer* L, size_t* total) {
    int idx = 0;
    size_t off = 0;
    auto add = [&](int cin, int cout, int level) {
        Layer l;
        l.cin = cin;
        l.cin_p = (cin + 31) / 32 * 32;
        l.cout = cout;
        l.level = level;
        l.w_off = off;
        off += (size_t)9 * cout * l.cin_p;
        l.b_off = off;
        off += cout;
        L[idx++] = l;
    };
    int c = 5;
    for (int i = 0; i < 4; ++i) {
        add(c, LEVEL_CH[i], i);
        add(LEVEL_CH[i], LEVEL_CH[i], i);
        c = LEVEL_CH[i];
    }
    for (int i = 2; i >= 0; --i) {
        add(c + LEVEL_CH[i], LEVEL_CH[i], i);
        add(LEVEL_CH[i], LEVEL_CH[i], i);
        c = LEVEL_CH[i];
    }
    *total = off + 5 * 32 + 5;  // head
}

size_t param_count() {
    Layer L[NCONV];
    size_t t;
    build_layers(L, &t);
    return t;
}

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

// activation tensors, in elements (bf16), per batch element count B
struct Acts {
    size_t x0, conv_out[NCONV], pool[4], cat[3], head_dA;
    size_t total;  // bytes of one activation set
};

Acts act_layout(int B, int H, int W) {
    Acts a{};
    size_t off = 0;
    auto px = [&](int level) { return (size_t)B * (H >> level) * (W >> level); };
    auto take = [&](size_t elems) {
        size_t o = off;
        off = a256(off + elems * 2);
        return o;
    };
    Layer L[NCONV];
    size_t t;
    build_layers(L, &t);
    a.x0 = take(px(0) * 32);
    for (int i = 1; i < 4; ++i) a.pool[i] = take(px(i) * LEVEL_CH[i - 1]);
    for (int k = 0; k < NCONV; ++k) a.conv_out[k] = take(px(L[k].level) * L[k].cout);
    for (int i = 0; i < 3; ++i) a.cat[i] = take(px(i) * (LEVEL_CH[i] + LEVEL_CH[i + 1]));
    a.head_dA = take(px(0) * 32);
    a.total = off;
    return a;
}

}  // namespace

struct sur_net {
    int B, H, W;
    Layer L[NCONV];
    size_t P;
    float *master, *grad, *m1, *m2;
    bf16 *wb, *wf;
    char* work;
    Acts fwd, bwd;  // activations and their gradients (same layout, two copies)
    float* dpred;   // [M][5]
    float* scal;    // loss accumulator etc.
    hipStream_t st;
    float mean[5], std[5], rstd[5], lw[5];
    int t = 0;
    int num_cu = 256;  // compute units of the device (work split of the weight gradient)
};

static size_t params_bytes(size_t P) {
    return a256(P * 4) * 4 + a256(P * 2) * 2;
}

static size_t workspace_bytes(int B, int H, int W) {
    Acts a = act_layout(B, H, W);
    size_t M = (size_t)B * H * W;
    return a.total * 2 + a256(M * 5 * 4) + 256;
}

static inline unsigned nb(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

static bf16* ACT(sur_net* h, bool grad, size_t off) { return (bf16*)(h->work + (grad ? h->fwd.total : 0) + off); }

static void conv_fwd(sur_net* h, int k, const bf16* in, bf16* out, bool act, int B) {
    const Layer& l = h->L[k];
    int Hl = h->H >> l.level, Wl = h->W >> l.level;
    launch_conv(h->st, in, h->wb + l.w_off, h->master + l.b_off, out, B, Hl, Wl, l.cin_p, l.cout, act);
}

// the input of conv layer k in the forward sequence
static const bf16* conv_input(sur_net* h, int k, bool grad) {
    // enc: 0:x0 1:out0 2:pool1 3:out2 4:pool2 5:out4 6:pool3 7:out6
    // dec: 8:cat2 9:out8 10:cat1 11:out10 12:cat0 13:out12
    Acts& a = h->fwd;
    switch (k) {
        case 0: return ACT(h, grad, a.x0);
        case 2: return ACT(h, grad, a.pool[1]);
        case 4: return ACT(h, grad, a.pool[2]);
        case 6: return ACT(h, grad, a.pool[3]);
        case 8: return ACT(h, grad, a.cat[2]);
        case 10: return ACT(h, grad, a.cat[1]);
        case 12: return ACT(h, grad, a.cat[0]);
        default: return ACT(h, grad, a.conv_out[k - 1]);
    }
}

static void forward(sur_net* h, int B) {
    Acts& a = h->fwd;
    for (int lv = 0; lv < 4; ++lv) {
        if (lv > 0) {
            int Hs = h->H >> (lv - 1), Ws = h->W >> (lv - 1), C = LEVEL_CH[lv - 1];
            hipLaunchKernelGGL(k_pool2, dim3(nb((long long)B * (Hs / 2) * (Ws / 2) * (C / 8))), dim3(256), 0, h->st,
                               ACT(h, false, a.conv_out[2 * lv - 1]), ACT(h, false, a.pool[lv]), B, Hs, Ws, C);
        }
        conv_fwd(h, 2 * lv, conv_input(h, 2 * lv, false), ACT(h, false, a.conv_out[2 * lv]), true, B);
        conv_fwd(h, 2 * lv + 1, conv_input(h, 2 * lv + 1, false), ACT(h, false, a.conv_out[2 * lv + 1]), true, B);
    }
    int prev = 7;
    for (int i = 2; i >= 0; --i) {
        int k = 8 + 2 * (2 - i);
        int Hl = h->H >> i, Wl = h->W >> i, Ca = h->L[prev].cout, Cs = LEVEL_CH[i];
        hipLaunchKernelGGL(k_up2_concat, dim3(nb((long long)B * Hl * Wl * ((Ca + Cs) / 8))), dim3(256), 0, h->st,
                           ACT(h, false, a.conv_out[prev]), ACT(h, false, a.conv_out[2 * i + 1]),
                           ACT(h, false, a.cat[i]), B, Hl, Wl, Ca, Cs);
        conv_fwd(h, k, conv_input(h, k, false), ACT(h, false, a.conv_out[k]), true, B);
        conv_fwd(h, k + 1, conv_input(h, k + 1, false), ACT(h, false, a.conv_out[k + 1]), true, B);
        prev = k + 1;
    }
}

// backward through conv layer k: dOut (gradient of its output, in the
// gradient set) -> parameter gradients and, unless k == 0, the gradient of
// its input (written to the gradient set's input slot, overwriting)
static void conv_bwd(sur_net* h, int k, int B) {
    const Layer& l = h->L[k];
    Acts& a = h->fwd;
    int Hl = h->H >> l.level, Wl = h->W >> l.level;
    long long M = (long long)B * Hl * Wl;
    bf16* dOut = ACT(h, true, a.conv_out[k]);
    hipLaunchKernelGGL(k_leaky_bwd, dim3(nb(M * l.cout / 8)), dim3(256), 0, h->st, ACT(h, false, a.conv_out[k]), dOut,
                       M * l.cout / 8);
    launch_wgrad(h->st, conv_input(h, k, false), (const bf16*)dOut, h->grad + l.w_off, B, Hl, Wl, l.cin_p, l.cout,
                 h->num_cu);
    const unsigned nbias = (unsigned)std::min<long long>(1024, std::max<long long>(1, M / 512));
    hipLaunchKernelGGL(k_bias_grad, dim3(nbias), dim3(256), 0, h->st, (const bf16*)dOut, h->grad + l.b_off, M, l.cout);
    if (k == 0) return;
    hipLaunchKernelGGL(k_flip, dim3(nb(9ll * l.cin_p * l.cout)), dim3(256), 0, h->st, h->wb + l.w_off,
                       h->wf + l.w_off, l.cin_p, l.cout);
    bf16* dIn = (bf16*)conv_input(h, k, true);
    launch_conv(h->st, (const bf16*)dOut, h->wf + l.w_off, nullptr, dIn, B, Hl, Wl, l.cout, l.cin_p, false);
}

static void backward(sur_net* h, int B) {
    Acts& a = h->fwd;
    // head gradient dA was written into the gradient of conv_out[13] by k_head
    int prevk = 13;
    for (int i = 0; i <= 2; ++i) {
        int k = 8 + 2 * (2 - i);  // dec{i}a; dec{i}b = k + 1
        conv_bwd(h, k + 1, B);      // writes grad of conv_out[k]
        conv_bwd(h, k, B);          // writes grad of cat[i]
        int Hl = h->H >> i, Wl = h->W >> i;
        int src = k - 1 == 7 ? 7 : k - 1;  // producer of the upsampled part
        int Ca = h->L[src].cout, Cs = LEVEL_CH[i];
        // dA -> gradient of the producer's output; dS -> gradient of the skip,
        // kept aside in the skip's own gradient slot for the encoder pass
        hipLaunchKernelGGL(k_up2_concat_bwd,
                           dim3(nb((long long)B * (Hl / 2) * (Wl / 2) * (Ca / 8) + (long long)B * Hl * Wl * (Cs / 8))), dim3(256), 0,
                           h->st, (const bf16*)ACT(h, true, a.cat[i]), ACT(h, true, a.conv_out[src]),
                           ACT(h, true, a.conv_out[2 * i + 1]), B, Hl, Wl, Ca, Cs);
        prevk = src;
    }
    (void)prevk;
    // encoder, deepest first; the skip gradient of level i already sits in
    // grad(conv_out[2i+1]) and the pooled path adds into it
    for (int lv = 3; lv >= 0; --lv) {
        conv_bwd(h, 2 * lv + 1, B);
        conv_bwd(h, 2 * lv, B);
        if (lv > 0) {
            int Hs = h->H >> (lv - 1), Ws = h->W >> (lv - 1), C = LEVEL_CH[lv - 1];
            hipLaunchKernelGGL(k_pool2_bwd, dim3(nb((long long)B * Hs * Ws * (C / 8))), dim3(256), 0, h->st,
                               (const bf16*)ACT(h, true, a.pool[lv]), ACT(h, true, a.conv_out[2 * lv - 1]), B, Hs,
                               Ws, C, 1);
        }
    }
}

extern "C" {

const char* sur_last_error(void) { return g_err.c_str(); }
size_t sur_param_count(void) { return param_count(); }
size_t sur_param_bytes(void) { return params_bytes(param_count()); }
size_t sur_workspace_bytes(int B, int H, int W) {
    if (B < 1 || H < 8 || W < 8 || (H % 8) || (W % 8)) return 0;
    return workspace_bytes(B, H, W);
}

int sur_create(int B, int H, int W, void* params, size_t pbytes, void* work, size_t wbytes, void* stream,
               sur_handle* out) {
    if (!out) return fail(-1, "null output");
    *out = nullptr;
    if (B < 1 || H < 8 || W < 8 || (H % 8) || (W % 8)) return fail(-1, "B >= 1, H and W multiples of 8");
    size_t P = param_count();
    if (!params || pbytes < params_bytes(P)) return fail(-2, "parameter block too small");
    if (!work || wbytes < workspace_bytes(B, H, W)) return fail(-2, "workspace too small");
    sur_net* h = new (std::nothrow) sur_net();
    if (h) {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            h->num_cu = ncu;
    }
    if (!h) return fail(-2, "host allocation failed");
    h->B = B;
    h->H = H;
    h->W = W;
    size_t t;
    build_layers(h->L, &t);
    h->P = P;
    char* p = (char*)params;
    h->master = (float*)p;
    p += a256(P * 4);
    h->grad = (float*)p;
    p += a256(P * 4);
    h->m1 = (float*)p;
    p += a256(P * 4);
    h->m2 = (float*)p;
    p += a256(P * 4);
    h->wb = (bf16*)p;
    p += a256(P * 2);
    h->wf = (bf16*)p;
    h->work = (char*)work;
    h->fwd = act_layout(B, H, W);
    h->dpred = (float*)(h->work + 2 * h->fwd.total);
    h->scal = (float*)(h->work + 2 * h->fwd.total + a256((size_t)B * H * W * 5 * 4));
    h->st = (hipStream_t)stream;
    for (int c = 0; c < 5; ++c) h->mean[c] = 0.f, h->std[c] = 1.f, h->rstd[c] = 1.f, h->lw[c] = 1.f;
    *out = h;
    return 0;
}

int sur_destroy(sur_handle h) {
    if (!h) return fail(-1, "null handle");
    delete h;
    return 0;
}

int sur_set_params(sur_handle h, const float* host) {
    if (!h || !host) return fail(-1, "null argument");
    HIP_TRY(hipMemcpyAsync(h->master, host, h->P * 4, hipMemcpyHostToDevice, h->st));
    hipLaunchKernelGGL(k_to_bf16, dim3(nb(h->P)), dim3(256), 0, h->st, h->master, h->wb, (long long)h->P);
    hipLaunchKernelGGL(k_fill, dim3(nb(h->P)), dim3(256), 0, h->st, h->m1, (long long)h->P, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(nb(h->P)), dim3(256), 0, h->st, h->m2, (long long)h->P, 0.f);
    HIP_TRY(hipStreamSynchronize(h->st));
    h->t = 0;
    return 0;
}

int sur_get_params(sur_handle h, float* host) {
    if (!h || !host) return fail(-1, "null argument");
    HIP_TRY(hipMemcpyAsync(host, h->master, h->P * 4, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(hipStreamSynchronize(h->st));
    return 0;
}

int sur_get_grads(sur_handle h, float* host) {
    if (!h || !host) return fail(-1, "null argument");
    HIP_TRY(hipMemcpyAsync(host, h->grad, h->P * 4, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(hipStreamSynchronize(h->st));
    return 0;
}

int sur_get_layer_tensor(sur_handle h, int k, int which, float* host) {
    if (!h || !host) return fail(-1, "null argument");
    if (k < 0 || k >= NCONV) return fail(-1, "layer index outside 0..13");
    if (which < 0 || which > 2) return fail(-1, "which must be 0 (input), 1 (output) or 2 (output gradient)");
    const Layer& l = h->L[k];
    const size_t px = (size_t)h->B * (h->H >> l.level) * (h->W >> l.level);
    const size_t n = px * (which == 0 ? l.cin_p : l.cout);
    const bf16* src = which == 0 ? conv_input(h, k, false) : ACT(h, which == 2, h->fwd.conv_out[k]);
    std::vector<uint16_t> raw(n);
    HIP_TRY(hipMemcpyAsync(raw.data(), src, n * 2, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(hipStreamSynchronize(h->st));
    for (size_t i = 0; i < n; ++i) {  // bf16 is the upper half of an FP32
        uint32_t u = (uint32_t)raw[i] << 16;
        std::memcpy(host + i, &u, 4);
    }
    return 0;
}

int sur_set_normalization(sur_handle h, const float* mean5, const float* std5, const float* rstd5) {
    if (!h || !mean5 || !std5 || !rstd5) return fail(-1, "null argument");
    for (int c = 0; c < 5; ++c) {
        if (!(std5[c] > 0.f) || !(rstd5[c] > 0.f)) return fail(-1, "scales must be positive");
        h->mean[c] = mean5[c];
        h->std[c] = std5[c];
        h->rstd[c] = rstd5[c];
    }
    return 0;
}

int sur_set_loss_weights(sur_handle h, const float* w5) {
    if (!h || !w5) return fail(-1, "null argument");
    float sum = 0.f;
    for (int c = 0; c < 5; ++c) {
        if (!(w5[c] >= 0.f) || !(w5[c] < 1e30f)) return fail(-1, "weights must be finite and >= 0");
        sum += w5[c];
    }
    if (!(sum > 0.f)) return fail(-1, "at least one weight must be positive");
    for (int c = 0; c < 5; ++c) h->lw[c] = w5[c];
    return 0;
}

static void pack(sur_net* h, int b, const float* x) {
    hipLaunchKernelGGL(k_pack, dim3(nb((long long)b * h->H * h->W)), dim3(256), 0, h->st, x,
                       ACT(h, false, h->fwd.x0), b, h->H, h->W, h->mean[0], h->mean[1], h->mean[2], h->mean[3],
                       h->mean[4], h->std[0], h->std[1], h->std[2], h->std[3], h->std[4]);
}

static HeadArgs head_args(sur_net* h, int b) {
    HeadArgs ha;
    for (int c = 0; c < 5; ++c) ha.rstd[c] = h->rstd[c], ha.lw[c] = h->lw[c];
    ha.inv_count = 1.f / (float)((double)b * h->H * h->W * 5);
    return ha;
}

int sur_forward(sur_handle h, int b, const float* x, double* out) {
    if (!h || !x || b < 1 || b > h->B) return fail(-1, "bad arguments");
    pack(h, b, x);
    forward(h, b);
    size_t head = h->P - 165;
    hipLaunchKernelGGL(k_head, dim3(nb((long long)b * h->H * h->W)), dim3(256), 0, h->st,
                       (const bf16*)ACT(h, false, h->fwd.conv_out[13]), h->master + head, h->master + head + 160, x,
                       (const float*)nullptr, h->dpred, (bf16*)nullptr, out, h->scal, h->grad + head + 160, b, h->H,
                       h->W, head_args(h, b));
    HIP_TRY(hipGetLastError());
    return 0;
}

int sur_gradients(sur_handle h, int b, const float* x, const float* y, float* loss) {
    if (!h || !x || !y || b < 1 || b > h->B) return fail(-1, "bad arguments");
    hipLaunchKernelGGL(k_fill, dim3(nb(h->P)), dim3(256), 0, h->st, h->grad, (long long)h->P, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, h->st, h->scal, 4ll, 0.f);
    pack(h, b, x);
    forward(h, b);
    size_t head = h->P - 165;
    long long M = (long long)b * h->H * h->W;
    const bf16* A = ACT(h, false, h->fwd.conv_out[13]);
    hipLaunchKernelGGL(k_head, dim3(nb(M)), dim3(256), 0, h->st, A, h->master + head, h->master + head + 160, x, y,
                       h->dpred, ACT(h, true, h->fwd.conv_out[13]), (double*)nullptr, h->scal,
                       h->grad + head + 160, b, h->H, h->W, head_args(h, b));
    const unsigned nhead = (unsigned)std::min<long long>(1024, std::max<long long>(1, M / 256));
    hipLaunchKernelGGL(k_head_wgrad, dim3(nhead), dim3(256), 0, h->st, A, (const float*)h->dpred, h->grad + head, M);
    backward(h, b);
    HIP_TRY(hipGetLastError());
    float l = 0.f;
    HIP_TRY(hipMemcpyAsync(&l, h->scal, 4, hipMemcpyDeviceToHost, h->st));
    HIP_TRY(hipStreamSynchronize(h->st));
    if (loss) *loss = l;
    return 0;
}

int sur_train_step(sur_handle h, int b, const float* x, const float* y, float lr, float* loss) {
    int rc = sur_gradients(h, b, x, y, loss);
    if (rc) return rc;
    h->t += 1;
    float c1 = 1.f - powf(0.9f, (float)h->t), c2 = 1.f - powf(0.999f, (float)h->t);
    hipLaunchKernelGGL(k_adam, dim3(nb(h->P)), dim3(256), 0, h->st, h->master, h->grad, h->m1, h->m2, h->wb,
                       (long long)h->P, lr, c1, c2);
    HIP_TRY(hipGetLastError());
    return 0;
}

static uint16_t host_bf16(float f) {  // round to nearest even
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static float host_f32(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

int sur_conv_check(int op, int B, int H, int W, int Cin, int Cout, const float* X, const float* Wt,
                   const float* dY, float* out) {
    if (op < 0 || op > 2 || B < 1 || H < 1 || W < 1 || Cin % 32 || Cout % 32 || !X || !Wt || !out ||
        (op > 0 && !dY))
        return fail(-1, "bad arguments");
    const size_t M = (size_t)B * H * W, nx = M * Cin, nw = 9ull * Cin * Cout, ny = M * Cout;
    std::vector<uint16_t> hx(nx), hw(nw), hy(ny);
    for (size_t i = 0; i < nx; ++i) hx[i] = host_bf16(X[i]);
    for (size_t i = 0; i < nw; ++i) hw[i] = host_bf16(Wt[i]);
    if (dY)
        for (size_t i = 0; i < ny; ++i) hy[i] = host_bf16(dY[i]);
    bf16 *dx = nullptr, *dw = nullptr, *dwf = nullptr, *dy = nullptr, *dout = nullptr;
    float *dbias = nullptr, *dgw = nullptr;
    hipError_t e = hipMalloc(&dx, nx * 2);
    if (e == hipSuccess) e = hipMalloc(&dw, nw * 2);
    if (e == hipSuccess) e = hipMalloc(&dwf, nw * 2);
    if (e == hipSuccess) e = hipMalloc(&dy, ny * 2);
    if (e == hipSuccess) e = hipMalloc(&dout, (nx > ny ? nx : ny) * 2);
    if (e == hipSuccess) e = hipMalloc(&dbias, Cout * 4);
    if (e == hipSuccess) e = hipMalloc(&dgw, nw * 4);
    if (e == hipSuccess) e = hipMemcpy(dx, hx.data(), nx * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dw, hw.data(), nw * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess && dY) e = hipMemcpy(dy, hy.data(), ny * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(dbias, 0, Cout * 4);
    if (e == hipSuccess) e = hipMemset(dgw, 0, nw * 4);
    if (e == hipSuccess) {
        if (op == 0) {
            launch_conv(0, dx, dw, dbias, dout, B, H, W, Cin, Cout, false);
        } else if (op == 1) {
            hipLaunchKernelGGL(k_flip, dim3(nb((long long)nw)), dim3(256), 0, 0, dw, dwf, Cin, Cout);
            launch_conv(0, dy, dwf, nullptr, dout, B, H, W, Cout, Cin, false);
        } else {
            launch_wgrad(0, dx, dy, dgw, B, H, W, Cin, Cout, 256);
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) {
        if (op == 2) {
            e = hipMemcpy(out, dgw, nw * 4, hipMemcpyDeviceToHost);
        } else {
            size_t n = op == 0 ? ny : nx;
            std::vector<uint16_t> ho(n);
            e = hipMemcpy(ho.data(), dout, n * 2, hipMemcpyDeviceToHost);
            for (size_t i = 0; i < n; ++i) out[i] = host_f32(ho[i]);
        }
    }
    for (void* q : {(void*)dx, (void*)dw, (void*)dwf, (void*)dy, (void*)dout, (void*)dbias, (void*)dgw})
        if (q) (void)hipFree(q);
    if (e != hipSuccess) return fail(-3, hipGetErrorString(e));
    return 0;
}

int sur_mfma_check(const float* A, const float* B, float* D) {
    if (!A || !B || !D) return fail(-1, "null argument");
    std::vector<bf16> a(512), b(512);
    for (int i = 0; i < 512; ++i) {
        a[i] = (bf16)A[i];
        b[i] = (bf16)B[i];
    }
    bf16 *da = nullptr, *db = nullptr;
    float* dd = nullptr;
    HIP_TRY(hipMalloc(&da, 1024));
    HIP_TRY(hipMalloc(&db, 1024));
    HIP_TRY(hipMalloc(&dd, 1024));
    HIP_TRY(hipMemcpy(da, a.data(), 1024, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(db, b.data(), 1024, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_mfma_check, dim3(1), dim3(64), 0, 0, da, db, dd);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpy(D, dd, 1024, hipMemcpyDeviceToHost));
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dd);
    return 0;
}

}  // extern "C"
