// Merged launches of a tick whose requests all belong to the FP32 buckets
// that take the secular core (ranks up to 64): one launch per phase covers
// every bucket, so the tick is a chain of kernels on one stream
//   upload -> projection pass 1 -> pass 2 -> cores -> V rotations (and the
//          U plan) -> U rotations
// instead of one chain per bucket on parallel lanes.  The merged launch of a
// phase gives each bucket a range of its blocks; the work of a block is the
// same code (and the same bits) as in the bucket's own launch.  The U
// rotations are planned on the device after the cores: only the requests
// whose append was not applied to W (deferred U) rotate U, and the plan
// lists exactly their row blocks, so the U launch has a fixed grid that
// loops over the planned blocks.
#pragma once
#include "isvd_update.h"

namespace isvd {

constexpr int kChainMax = 4;          // buckets 8, 16, 32, 64
constexpr int kChainRowsU = 512;      // U rows per block of the planned U rotations
constexpr int kChainUGrid = 2048;     // blocks of the U-rotation launch (loop past that)
constexpr int kChainMaxReqs = 16384; // requests of a merged tick at most

// The request lists of one merged launch, one entry per bucket, in launch
// order; bucket q owns blocks [begin[q], begin[q + 1]).  tbl[q]: request and
// tile of each of the bucket's blocks (projections, V rotations), written by
// the host with the records; unused by the cores (one block per request) and
// the planned U rotations.
struct MultiGroup {
    int n = 0;
    int kc[kChainMax];
    const Req* reqs[kChainMax];
    const BlockRef* tbl[kChainMax];
    int nreq[kChainMax];
    int begin[kChainMax + 1];
};

// ints of the device plan of a tick's U rotations for up to `reqs` requests:
// [0] planned blocks, [1, reqs + 2) block prefix, then one code per request
__host__ __device__ constexpr size_t chain_plan_ints(int reqs) { return 2 + 2 * (size_t)reqs + 2; }

// bucket of merged block b (blockIdx.x unless given) and its block in the bucket
__device__ inline int chain_pick(const MultiGroup& mg, int* bid, int b = -1) {
    if (b < 0) b = (int)blockIdx.x;
    int q = 0;
    while (q + 1 < mg.n && b >= mg.begin[q + 1]) ++q;
    *bid = b - mg.begin[q];
    return q;
}

__host__ __device__ constexpr int chain_proj_lds() {
    return proj_lds_doubles<8>() > proj_lds_doubles<16>()
               ? (proj_lds_doubles<8>() > proj_lds_doubles<32>() ? proj_lds_doubles<8>() : proj_lds_doubles<32>())
               : (proj_lds_doubles<16>() > proj_lds_doubles<32>() ? proj_lds_doubles<16>() : proj_lds_doubles<32>());
}

template <int PASS>
__global__ void __launch_bounds__(kThreads) k_proj_chain(MultiGroup mg) {
    constexpr int L = chain_proj_lds() > proj_lds_doubles<64>() ? chain_proj_lds() : proj_lds_doubles<64>();
    __shared__ double lds[L];
    int bid;
    const int q = chain_pick(mg, &bid);
    const BlockRef br = mg.tbl[q][bid];
    const Req* rq = mg.reqs[q] + br.req;
    switch (mg.kc[q]) {
        case 8: proj_tile<float, 8, PASS>(rq, br.tile, lds); break;
        case 16: proj_tile<float, 16, PASS>(rq, br.tile, lds); break;
        case 32: proj_tile<float, 32, PASS>(rq, br.tile, lds); break;
        default: proj_tile<float, 64, PASS>(rq, br.tile, lds); break;
    }
}

// dynamic LDS (doubles) of the merged core launch: the widest bucket's
__host__ __device__ constexpr size_t chain_core_lds() { return core_lds_doubles<64, false>(); }

__global__ void __launch_bounds__(kSecCoreThreads) __attribute__((amdgpu_waves_per_eu(3))) k_core_chain(MultiGroup mg) {
    int bid;
    const int q = chain_pick(mg, &bid);
    switch (mg.kc[q]) {
        case 8: core_block<float, 8>(mg.reqs[q] + bid); break;
        case 16: core_block<float, 16>(mg.reqs[q] + bid); break;
        case 32: core_block<float, 32>(mg.reqs[q] + bid); break;
        default: core_block<float, 64>(mg.reqs[q] + bid); break;
    }
}

// Plan of the U rotations: request g (over the buckets in order) rotates U
// in ceil(m / kChainRowsU) blocks unless its core skipped it or applied its
// append to W.  Writes the planned blocks, their prefix over the requests
// and the request codes (bucket << 24 | index).  Run by one block of
// kThreads after the cores (the last block of the V launch): each thread
// takes a run of requests, counts their blocks, and after an exclusive scan
// over the block writes their prefix entries.
__device__ inline void chain_plan_block(const MultiGroup& mg, int* __restrict__ plan) {
    __shared__ int wsum[kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int G = 0;
    for (int q = 0; q < mg.n; ++q) G += mg.nreq[q];
    int* prefix = plan + 1;
    int* code = plan + 2 + G;
    const int per = (G + kThreads - 1) / kThreads;
    const int g0 = tid * per;
    auto blocks_of = [&](int g, int* cd) -> int {
        int q = 0, base = 0;
        while (g >= base + mg.nreq[q]) {
            base += mg.nreq[q];
            ++q;
        }
        const int ri = g - base;
        const Req& rq = mg.reqs[q][ri];
        const ISVD_GLOBAL ReqScratch* rs = gmem(rq.rs);
        *cd = (q << 24) | ri;
        return (rs->skip || rs->deferred) ? 0 : (int)((rq.m + kChainRowsU - 1) / kChainRowsU);
    };
    int local = 0;
    for (int i = 0; i < per; ++i) {
        int cd;
        if (g0 + i < G) local += blocks_of(g0 + i, &cd);
    }
    // exclusive prefix of `local` over the block: within the wave, then over the waves
    int incl = local;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += wsum[w];
    int run = wbase + incl - local;
    for (int i = 0; i < per; ++i) {
        const int g = g0 + i;
        if (g >= G) break;
        int cd;
        const int bl = blocks_of(g, &cd);
        prefix[g] = run;
        code[g] = cd;
        run += bl;
    }
    if (tid == kThreads - 1) {
        plan[0] = run;
        prefix[G] = run;
    }
}

// V tiles (part 2) of every bucket, kRotRowsV rows per block, after a first
// block that writes the plan of the U rotations (the cores have run), so
// that the plan overlaps the V tiles.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
k_rotv_chain(MultiGroup mg, int* __restrict__ plan) {
    if (blockIdx.x == 0) {
        chain_plan_block(mg, plan);
        return;
    }
    int bid;
    const int q = chain_pick(mg, &bid, (int)blockIdx.x - 1);
    const BlockRef br = mg.tbl[q][bid];
    const Req* rq = mg.reqs[q] + br.req;
    const int tile = br.tile;
    switch (mg.kc[q]) {
        case 8: rotate_mfma_t_block<8, kRotRowsV, 1, true>(rq, tile, 2); break;
        case 16: rotate_mfma_t_block<16, kRotRowsV, 1, true>(rq, tile, 2); break;
        case 32: rotate_mfma_t_block<32, kRotRowsV, 1, true>(rq, tile, 2); break;
        default: rotate_mfma_t_block<64, kRotRowsV, 1, true>(rq, tile, 2); break;
    }
}

// The planned U-rotation blocks: a fixed grid, each block taking planned
// blocks blockIdx.x, blockIdx.x + gridDim.x, ...
__global__ void __launch_bounds__(kThreads) k_rotu_chain(MultiGroup mg, const int* __restrict__ plan) {
    int G = 0;
    for (int q = 0; q < mg.n; ++q) G += mg.nreq[q];
    const int total = plan[0];
    const int* prefix = plan + 1;
    const int* code = plan + 2 + G;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int g = find_req(prefix, G, t);
        const int c = code[g];
        const int q = c >> 24, ri = c & 0xFFFFFF;
        const Req* rq = mg.reqs[q] + ri;
        const int tile = t - prefix[g];
        switch (mg.kc[q]) {
            case 8: rotate_mfma_t_block<8, kChainRowsU, 1, true>(rq, tile, 1); break;
            case 16: rotate_mfma_t_block<16, kChainRowsU, 1, true>(rq, tile, 1); break;
            case 32: rotate_mfma_t_block<32, kChainRowsU, 1, true>(rq, tile, 1); break;
            default: rotate_mfma_t_block<64, kChainRowsU, 1, true>(rq, tile, 1); break;
        }
        __syncthreads();   // the block's LDS (projection data) is reused by its next planned block
    }
}

}  // namespace isvd
