// batch.h -- one launch per kernel class for many independent solvers.
//
// A batch holds independent seeds (grids of any size, their own physical
// parameters) that step in lockstep.  Each kernel class runs as one launch
// over a global list of (seed, tile) work items, seed by seed and row by row:
// the list is cut into one band per XCD and the workgroups of an XCD take the
// items of their band in turn (batch_span), so neighbouring tiles of a seed
// run together under one L2.  The grid is a launch parameter: fewer
// workgroups than items make it persistent (each loops over its items), as
// many give one item per workgroup.  Per node the
// arithmetic is the single-solver kernels' (same device functions), so every
// member evolves bit for bit as it would alone.
#pragma once

#include "kernels.h"

namespace dlb {

// A member's arrays are byte offsets into the batch's state buffer, whose
// base the kernels take as an argument: pointers derived from a kernel
// argument are known to address global memory, so the compiler emits global
// loads and stores, where pointers read from memory would give generic
// (flat) ones.
struct SeedDesc {
    KParams kp;
    size_t pop[2];
    size_t flow[2];
    size_t hist;
    int hist_valid;
    int tile0;      // first node tile of this seed in the node-kernel work list
    int node_nbx;   // node tiles per row (tile width x 256/width nodes, set per batch)
    int tb0[2];     // first extended tile in the fused-flow work list, K = 3 / K = 5
    int tb_nbx[2];  // extended tiles per row, K = 3 / K = 5
};

// seed owning work item `item`; list -1 = node tiles, 0/1 = fused tiles K = 3/5
__device__ __forceinline__ int seed_of(const SeedDesc* __restrict__ d, int count, int item, int list) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int start = list < 0 ? d[mid].tile0 : d[mid].tb0[list];
        if (start <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// node (x, y) of this thread in node tile t of a seed: tiles of 2^tw_log2
// columns by BLOCK >> tw_log2 rows, one node per thread
__device__ __forceinline__ void batch_node(const SeedDesc& sd, int t, int tw_log2, int& x, int& y) {
    x = ((t % sd.node_nbx) << tw_log2) + (threadIdx.x & ((1 << tw_log2) - 1));
    y = (t / sd.node_nbx) * (BLOCK >> tw_log2) + (threadIdx.x >> tw_log2);
}

// Items of a batch launch taken by this block: the work list is
// cut into 8 contiguous bands, one per XCD (block b runs on XCD b mod 8),
// and the blocks of one XCD interleave over their band, so that tiles
// sharing halo rows or streaming targets (the next tile row of the same
// seed) run at the same time under one L2.  A grid that is not a multiple
// of 8 blocks interleaves over the whole list.  Items rise within a block.
struct BatchSpan {
    int beg, end, stride;
};
__device__ __forceinline__ BatchSpan batch_span(int total) {
    if (gridDim.x % 8 == 0) {
        const int band = (total + 7) / 8, x = (int)(blockIdx.x % 8);
        return {x * band + (int)(blockIdx.x / 8), min((x + 1) * band, total), (int)(gridDim.x / 8)};
    }
    return {(int)blockIdx.x, total, (int)gridDim.x};
}

template <class CF, bool NS, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_pct_batch(char* __restrict__ base, const SeedDesc* __restrict__ d,
                                                     int count, int total, int cur, int fcur, int tw_log2) {
    using S = typename CF::S;
    using H = typename CF::H;
    const BatchSpan w = batch_span(total);
    int s = w.beg < w.end ? seed_of(d, count, w.beg, -1) : 0;
    for (int item = w.beg; item < w.end; item += w.stride) {
        while (s + 1 < count && d[s + 1].tile0 <= item) ++s;
        const SeedDesc& sd = d[s];
        int x, y;
        batch_node(sd, item - sd.tile0, tw_log2, x, y);
        if (x < sd.kp.nx && y < sd.kp.ny)
            pct_node<CF, NS, WALLS>(sd.kp, (const S*)(base + sd.pop[cur]), (S*)(base + sd.pop[1 - cur]),
                                    (const S*)(base + sd.flow[fcur]), (H*)(base + sd.hist), sd.hist_valid, x, y);
    }
}

template <class CF, bool WALLS>
__global__ __launch_bounds__(BLOCK) void k_flow_batch(char* __restrict__ base, const SeedDesc* __restrict__ d,
                                                      int count, int total, int fcur, int tw_log2) {
    using S = typename CF::S;
    using H = typename CF::H;
    const BatchSpan w = batch_span(total);
    int s = w.beg < w.end ? seed_of(d, count, w.beg, -1) : 0;
    for (int item = w.beg; item < w.end; item += w.stride) {
        while (s + 1 < count && d[s + 1].tile0 <= item) ++s;
        const SeedDesc& sd = d[s];
        int x, y;
        batch_node(sd, item - sd.tile0, tw_log2, x, y);
        if (x < sd.kp.nx && y < sd.kp.ny)
            flow_step_node<CF, WALLS>(sd.kp, (const S*)(base + sd.flow[fcur]), (S*)(base + sd.flow[1 - fcur]),
                                      (const H*)(base + sd.hist), x, y);
    }
}

template <class CF, bool WALLS, int K>
__global__ __launch_bounds__(TbGeom<typename CF::T>::THREADS) void k_flow_tb_batch(char* __restrict__ base,
                                                                                  const SeedDesc* __restrict__ d,
                                                                                  int count, int total, int fcur) {
    using S = typename CF::S;
    using H = typename CF::H;
    constexpr int L = K == 5 ? 1 : 0;
    const BatchSpan w = batch_span(total);
    int s = w.beg < w.end ? seed_of(d, count, w.beg, L) : 0;
    for (int item = w.beg; item < w.end; item += w.stride) {
        while (s + 1 < count && d[s + 1].tb0[L] <= item) ++s;
        const SeedDesc& sd = d[s];
        const int t = item - sd.tb0[L];
        flow_fused_tile<CF, WALLS, K>(sd.kp, (const S*)(base + sd.flow[fcur]), (S*)(base + sd.flow[1 - fcur]),
                                      (const H*)(base + sd.hist), t % sd.tb_nbx[L], t / sd.tb_nbx[L]);
        __syncthreads();  // LDS of this tile is reused by the next
    }
}

}  // namespace dlb
