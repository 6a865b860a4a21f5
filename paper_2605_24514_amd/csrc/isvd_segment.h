// Segmented refresh launches: the A-form refreshes (Sec. 2.4.1) that one
// tick's policies fire run phase by phase, one launch per phase for all of
// them, instead of a chain of small launches per stream.  Job j of a launch
// owns blocks [begin[j], begin[j + 1]); a block runs the body of the
// per-stream kernel with the job's arguments and its block index within the
// job, so every stream gets bitwise the result of its own launches.  Most
// refresh phases of a serving-sized stream are one block (Cholesky, the
// Rayleigh-Ritz SVD) or a few dozen; a segmented launch gives the chip one
// block per stream instead of one stream at a time.
#pragma once
#include "isvd_refresh.h"

namespace isvd {

// job of block blockIdx.x: the largest j with begin[j] <= blockIdx.x (begin[0] = 0)
__device__ inline int seg_job(const int* __restrict__ begin, int njobs) {
    const int bx = (int)blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= bx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct SjStart {
    float* X;
    const float* V;
    int* flags;
    int64_t n;
    uint64_t seed;
    int ldx, b, ldv, kw, ident;
};
struct SjGram {
    const float* Y;
    double* Gp;
    int64_t rows, rpb;
    int ldy, b;
};
struct SjGramSum {
    const double* Gp;
    double* G;
    int nparts, b;
};
struct SjChol {
    const double* G;
    double* R;
    float* RinvT;
    int* flag;
    int b;
};
struct SjNN {
    const float* A;
    const float* X;
    float* Y;
    int64_t lda, m, n;
    int ldy, b;
};
struct SjTN {
    const float* A;
    const float* Q;
    float* Zp;
    int64_t lda, m, n, rpc;
    int b, gx;   // column blocks of the job's grid (block = y gx + x)
};
struct SjTnSum {
    const float* Zp;
    float* Z;
    int64_t per_chunk, n;
    int nchunk, b, ldz;
};
struct SjSmallGemm {
    const double* A;
    const double* B;
    double* C;
    int b;
};
struct SjRot {
    const float* in;
    float* out;
    const float* Q;
    float* out2;
    int64_t rows;
    int ldi, ldo, kin;
};
struct SjSvd {
    const double* R;
    double* S;
    float* QU;
    float* QV;
    int* sweeps;
    int b, k, ldo;
};

__global__ void __launch_bounds__(256) k_seg_start(const SjStart* __restrict__ jobs, const int* __restrict__ begin,
                                                   int njobs) {
    const int j = seg_job(begin, njobs);
    const SjStart a = jobs[j];
    k_start_block_body<float>(a.X, a.ldx, a.n, a.b, a.V, a.ldv, a.kw, a.seed, a.ident, a.flags,
                              (int)blockIdx.x - begin[j], 0, 0);
}

__global__ void __launch_bounds__(kThreads) k_seg_gram(const SjGram* __restrict__ jobs, const int* __restrict__ begin,
                                                       int njobs) {
    const int j = seg_job(begin, njobs);
    const SjGram a = jobs[j];
    k_gram_mfma_body<float, false>(a.Y, a.ldy, a.rows, a.b, a.rpb, a.Gp, (int)blockIdx.x - begin[j], 0, 0);
}

__global__ void __launch_bounds__(256) k_seg_gram_sum(const SjGramSum* __restrict__ jobs,
                                                      const int* __restrict__ begin, int njobs) {
    const int j = seg_job(begin, njobs);
    const SjGramSum a = jobs[j];
    k_gram_sum_body(a.Gp, a.nparts, a.b, a.G, (int)blockIdx.x - begin[j], 0, 0);
}

// one block per job
__global__ void __launch_bounds__(kCholThreads) k_seg_chol(const SjChol* __restrict__ jobs) {
    const SjChol a = jobs[blockIdx.x];
    k_chol_inv_body<float>(a.G, a.b, a.R, a.RinvT, a.flag, 0, 0, 0);
}

template <int NB>
__global__ void __launch_bounds__(kThreads, 2) k_seg_nn(const SjNN* __restrict__ jobs, const int* __restrict__ begin,
                                                        int njobs) {
    const int j = seg_job(begin, njobs);
    const SjNN a = jobs[j];
    k_gemm_nn_mfma_body<2, NB, kNnChunk>(a.A, a.lda, a.X, a.Y, a.ldy, a.m, a.n, a.b, (int)blockIdx.x - begin[j],
                                         0, 0);
}

template <int NB>
__global__ void __launch_bounds__(kThreads, 2) k_seg_tn(const SjTN* __restrict__ jobs, const int* __restrict__ begin,
                                                        int njobs) {
    const int j = seg_job(begin, njobs);
    const SjTN a = jobs[j];
    const int t = (int)blockIdx.x - begin[j];
    k_gemm_tn_mfma_body<NB, kTnRows>(a.A, a.lda, a.Q, a.Zp, a.m, a.n, a.b, a.rpc, t % a.gx, t / a.gx, a.gx);
}

__global__ void __launch_bounds__(256) k_seg_tn_sum(const SjTnSum* __restrict__ jobs, const int* __restrict__ begin,
                                                    int njobs) {
    const int j = seg_job(begin, njobs);
    const SjTnSum a = jobs[j];
    k_tn_sum_body(a.Zp, a.nchunk, a.per_chunk, a.n, a.b, a.Z, a.ldz, (int)blockIdx.x - begin[j], 0, 0);
}

__global__ void __launch_bounds__(256) k_seg_small_gemm(const SjSmallGemm* __restrict__ jobs,
                                                        const int* __restrict__ begin, int njobs) {
    const int j = seg_job(begin, njobs);
    const SjSmallGemm a = jobs[j];
    k_small_gemm_body(a.A, a.B, a.C, a.b, (int)blockIdx.x - begin[j], 0, 0);
}

template <bool TILED_OUT>
__global__ void __launch_bounds__(kThreads) k_seg_rot(const SjRot* __restrict__ jobs, const int* __restrict__ begin,
                                                      int njobs) {
    const int j = seg_job(begin, njobs);
    const SjRot a = jobs[j];
    k_rotate_plain_body<float, 128, TILED_OUT>(a.in, a.ldi, a.out, a.ldo, a.rows, a.kin, a.Q, a.out2,
                                               (int)blockIdx.x - begin[j], 0, 0);
}

// one block per job
__global__ void __launch_bounds__(RRShape::NT) k_seg_svd(const SjSvd* __restrict__ jobs) {
    extern __shared__ double smem[];
    const SjSvd a = jobs[blockIdx.x];
    k_svd_small_noj_body<float>(a.R, a.b, a.k, a.S, a.QU, a.QV, a.ldo, a.sweeps, smem);
}

}  // namespace isvd
