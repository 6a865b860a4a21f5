// Refresh kernels: TruncatedSVD(A_t, k) (Algorithm 1 init and refresh,
// Section 2.4.1) by block subspace iteration on the dense A held in HBM.
//
//   X (n x b) orthonormal start: identity when b = n (the iteration is then
//   exact), else the current V_t completed by pseudo-random columns.
//   repeat q times:  Q = orth(A X);  X = orth(A^T Q)
//   Rayleigh-Ritz:   A X = Q_Y R_Y (CholQR2),  R_Y = W S H^T (FP64 Jacobi)
//                    U = Q_Y W[:, :k],  Sigma = S[:k],  V = X H[:, :k]
//
// orth() is CholQR2: Gram matrix in FP64 (products of the storage type
// accumulated in FP64, split over row chunks and summed in chunk order),
// Cholesky and triangular inverse in FP64 in one block, Y <- Y R^{-1},
// twice.  The small GEMMs here are plain LDS-tiled VALU code.
#pragma once
#include <algorithm>
#include "isvd_common.h"
#include "isvd_jacobi.h"

namespace isvd {

constexpr int kGemmRows = 64;
constexpr int kGemmK = 32;

// Y[m x b] = A[m x n] X[n x b]   (b <= 128)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_gemm_nn(const T* __restrict__ A, int64_t lda,
                                                      const T* __restrict__ X, int ldx,
                                                      T* __restrict__ Y, int ldy,
                                                      int64_t m, int64_t n, int b) {
    __shared__ T sA[kGemmRows][kGemmK + 1];
    __shared__ T sX[kGemmK][128];
    const int64_t r0 = (int64_t)blockIdx.x * kGemmRows;
    const int row = threadIdx.x % kGemmRows;
    const int cg = threadIdx.x / kGemmRows;   // 0..3
    T acc[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] = (T)0;
    for (int64_t c0 = 0; c0 < n; c0 += kGemmK) {
        for (int e = threadIdx.x; e < kGemmRows * kGemmK; e += kThreads) {
            int rr = e / kGemmK, cc = e % kGemmK;
            int64_t r = r0 + rr, c = c0 + cc;
            sA[rr][cc] = (r < m && c < n) ? A[r * lda + c] : (T)0;
        }
        for (int e = threadIdx.x; e < kGemmK * b; e += kThreads) {
            int cc = e / b, j = e % b;
            int64_t c = c0 + cc;
            sX[cc][j] = c < n ? X[c * ldx + j] : (T)0;
        }
        __syncthreads();
        for (int cc = 0; cc < kGemmK; ++cc) {
            T a = sA[row][cc];
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                int j = cg + 4 * q;
                if (j < b) acc[q] += a * sX[cc][j];
            }
        }
        __syncthreads();
    }
    int64_t r = r0 + row;
    if (r < m) {
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            int j = cg + 4 * q;
            if (j < b) Y[r * ldy + j] = acc[q];
        }
    }
}

// Zp[chunk][c][j] = sum over rows r of the chunk of A[r][c] Q[r][j]  (FP64 partials)
// grid: (ceil(n / 64), nchunks)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_gemm_tn_partial(const T* __restrict__ A, int64_t lda,
                                                              const T* __restrict__ Q, int ldq,
                                                              double* __restrict__ Zp,
                                                              int64_t m, int64_t n, int b,
                                                              int64_t rows_per_chunk) {
    __shared__ T sA[kGemmK][64 + 1];
    __shared__ T sQ[kGemmK][128];
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const int64_t ra = (int64_t)blockIdx.y * rows_per_chunk;
    const int64_t rb = min(m, ra + rows_per_chunk);
    const int col = threadIdx.x % 64;
    const int jg = threadIdx.x / 64;
    double acc[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] = 0.0;
    for (int64_t r0 = ra; r0 < rb; r0 += kGemmK) {
        for (int e = threadIdx.x; e < kGemmK * 64; e += kThreads) {
            int rr = e / 64, cc = e % 64;
            int64_t r = r0 + rr, c = c0 + cc;
            sA[rr][cc] = (r < rb && c < n) ? A[r * lda + c] : (T)0;
        }
        for (int e = threadIdx.x; e < kGemmK * b; e += kThreads) {
            int rr = e / b, j = e % b;
            int64_t r = r0 + rr;
            sQ[rr][j] = r < rb ? Q[r * ldq + j] : (T)0;
        }
        __syncthreads();
        for (int rr = 0; rr < kGemmK; ++rr) {
            double a = (double)sA[rr][col];
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                int j = jg + 4 * q;
                if (j < b) acc[q] += a * (double)sQ[rr][j];
            }
        }
        __syncthreads();
    }
    int64_t c = c0 + col;
    if (c < n) {
        double* out = Zp + ((int64_t)blockIdx.y * n + c) * b;
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            int j = jg + 4 * q;
            if (j < b) out[j] = acc[q];
        }
    }
}

// ---------------------------------------------------------------------------
// Matrix-core versions of the refresh products (b <= kMaxBlock columns).
// v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64 lane layout: A[l%16][l/16],
// B[l/16][l%16]; FP32 D[4(l/16)+r][l%16], FP64 D[4r+l/16][l%16].
typedef float mm_v4f __attribute__((ext_vector_type(4)));
typedef double mm_v4d __attribute__((ext_vector_type(4)));

// Y[m x b] = A[m x n] X[n x b], FP32 in and FP32 accumulation (b <= kMaxBlock).  A
// wave owns RB 16-row MFMA blocks and runs over all of n; a block's four
// waves share X, staged KCH rows at a time in double-buffered LDS, and each
// wave prefetches its next KCH columns of A into registers while the matrix
// cores work on the current ones (one barrier per chunk).  Per 16-column
// slab lane l loads one float4 of A per row block -- row l%16, columns
// k0 + 4 (l/16) + 0..3 -- and MFMA step s takes column k0 + 4 (l/16) + s, so
// the B operand is X[k0 + 4 (l/16) + s][16 q + l%16] from LDS.  X is n x b
// with leading dimension b.  lda % 4 == 0,
// and A's columns in [n, round4(n)) must hold finite values (they are read
// and multiplied by zero).
// Y may be A itself (ldy == lda): a wave reads all of its rows before it
// writes them.  grid ceil(m / (64 RB)).
constexpr int kStageLd = kMaxBlock + 4;   // LDS row stride: the four lane groups hit disjoint banks
// Copy of ROWS rows of a row-major FP32 matrix whose leading dimension
// equals its width `cols` (<= W), so the rows form one contiguous run of
// ROWS cols floats: thread t takes elements t, t + 256, ... of the run
// (coalesced loads at fixed offsets from one base) and stores them at LDS
// row stride kStageLd.  Elements past the end of the matrix are stored as
// zero; LDS columns in [cols, W) are left as they are.  The LDS offsets do
// not depend on the chunk and are computed once.
template <int ROWS, int W>
struct StageCopy {
    static constexpr int PER = (ROWS * W + kThreads - 1) / kThreads;
    int off[PER];
    float v[PER];
    __device__ void init(int cols) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + kThreads * i;
            off[i] = e < ROWS * cols ? (e / cols) * kStageLd + e % cols : -1;
        }
    }
    // run: first element of the chunk's rows; rem: elements left in the matrix from there
    __device__ void load(const float* __restrict__ run, int64_t rem) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + kThreads * i;
            v[i] = (off[i] >= 0 && e < rem) ? run[e] : 0.f;
        }
    }
    __device__ void store(float* __restrict__ lds) const {
#pragma unroll
        for (int i = 0; i < PER; ++i)
            if (off[i] >= 0) lds[off[i]] = v[i];
    }
};

constexpr int kNnChunk = 16;   // default columns of A per pipeline stage
template <int RB, int NB, int KCH = kNnChunk>
__device__ __attribute__((always_inline)) inline void k_gemm_nn_mfma_body(const float* A, int64_t lda,
                                                           const float* __restrict__ X,
                                                           float* Y, int ldy,
                                                           int64_t m, int64_t n, int b, const int bx_, const int by_,
    const int gx_) {
    typedef __attribute__((address_space(1))) const mm_v4f gc4;
    constexpr int SL = KCH / 16;                         // 16-column slabs per chunk
    constexpr int XW = 16 * NB;                                // staged columns of X
    __shared__ float sX[2][KCH * kStageLd];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = l >> 4, c16 = l & 15;
    const int64_t r0 = ((int64_t)bx_ * 4 + w) * (16 * RB);
    const int nch = (int)((n + KCH - 1) / KCH);
    StageCopy<KCH, XW> xn;
    xn.init(b);
    mm_v4f an[RB][SL];
    auto fetch = [&](int c) {
        xn.load(X + (int64_t)c * KCH * b, (n - (int64_t)c * KCH) * b);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) {
                const int64_t row = r0 + 16 * rb + c16;
                const int64_t kc = (int64_t)c * KCH + 16 * sl + 4 * g;
                // columns in [n, round4(n)) are read too: they meet zero rows of
                // the staged X, and A keeps them zero (finite) in its padding
                mm_v4f v = (mm_v4f){0.f, 0.f, 0.f, 0.f};
                if (row < m && kc < n) v = *(gc4*)(A + row * lda + kc);
                an[rb][sl] = v;
            }
    };
    auto stage = [&](int buf) { xn.store(sX[buf]); };
    mm_v4f acc[RB][NB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[rb][q] = (mm_v4f){0.f, 0.f, 0.f, 0.f};
    const bool active = r0 < m;
    fetch(0);
    stage(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        mm_v4f ac[RB][SL];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) ac[rb][sl] = an[rb][sl];
        if (c + 1 < nch) fetch(c + 1);
        if (active) {
            const float* xs = sX[c & 1];
            // B operands one slab ahead of the products that use them; the
            // scheduling barriers keep the compiler from pulling each read down
            // next to its use (which would expose the LDS latency)
            float xv[2][4][NB];
            auto read_slab = [&](int sl, float (&d)[4][NB]) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                    for (int q = 0; q < NB; ++q) d[s4][q] = xs[(16 * sl + 4 * g + s4) * kStageLd + 16 * q + c16];
            };
            read_slab(0, xv[0]);
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) {
                if (sl + 1 < SL) read_slab(sl + 1, xv[(sl + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int q = 0; q < NB; ++q)
                            acc[rb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[rb][sl][s4], xv[sl & 1][s4][q],
                                                                              acc[rb][q], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (c + 1 < nch) stage((c + 1) & 1);
        __syncthreads();
    }
    if (!active) return;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int col = 16 * q + c16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + 16 * rb + 4 * g + r;
                if (row < m && col < b) Y[row * ldy + col] = acc[rb][q][r];
            }
        }
}

template <int RB, int NB, int KCH = kNnChunk>
__global__ void __launch_bounds__(kThreads, 2) k_gemm_nn_mfma(const float* A, int64_t lda,
                                                           const float* __restrict__ X,
                                                           float* Y, int ldy,
                                                           int64_t m, int64_t n, int b) {
    k_gemm_nn_mfma_body<RB, NB, KCH>(A, lda, X, Y, ldy, m, n, b, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// Partials of Z = A^T Q (n x b, b <= kMaxBlock), computed as Z^T = Q^T A on the
// matrix cores (A operand Q^T, B operand A).  Block (x, y) covers columns
// [256 x, 256 x + 256) -- wave w the 64 from 256 x + 64 w -- over the rows
// of chunk y.  The four waves share the chunk's rows of Q, staged 32 at a
// time in double-buffered LDS; each wave prefetches its next 32 x 64 block
// of A into registers.  Per 4-row slab lane l loads one float4 of A -- row
// r0 + l/16, columns c0 + 4 (l%16) + 0..3 -- and feeds element j to the MFMA
// of column set j (columns c0 + 4 n + j).  FP32 accumulation; each lane
// stores its accumulators as they sit in the registers (b rounded to 16 floats per lane,
// coalesced), and k_tn_sum adds the chunks in FP64 and scatters them to Z.
// Q is m x b with leading dimension b; lda % 4 == 0.
constexpr int kTnCols = 256;
constexpr int kTnRows = 16;
constexpr int kTnDump = 4 * kMaxBlock * 64;   // floats per block of the partial dump
inline int64_t tn_chunks(int64_t m, int64_t n) {
    const int64_t ncb = (n + kTnCols - 1) / kTnCols;
    const int64_t want = (512 + ncb - 1) / ncb;
    return std::max<int64_t>(1, std::min<int64_t>(want, (m + 2 * kTnRows - 1) / (2 * kTnRows)));
}
template <int NB, int RCH = kTnRows>
__device__ __attribute__((always_inline)) inline void k_gemm_tn_mfma_body(const float* __restrict__ A, int64_t lda,
                                                           const float* __restrict__ Q,
                                                           float* __restrict__ Zp, int64_t m, int64_t n, int b,
                                                           int64_t rows_per_chunk, const int bx_, const int by_,
    const int gx_) {
    typedef __attribute__((address_space(1))) const mm_v4f gc4;
    constexpr int SLABS = RCH / 4;
    constexpr int QW = 16 * NB;
    __shared__ float sQ[2][RCH * kStageLd];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = l >> 4, c16 = l & 15;
    const int64_t cc = (int64_t)bx_ * kTnCols + 64 * w + 4 * c16;
    const int64_t ra = (int64_t)by_ * rows_per_chunk;
    const int64_t rb = min(m, ra + rows_per_chunk);
    const int nch = rb > ra ? (int)((rb - ra + RCH - 1) / RCH) : 0;
    StageCopy<RCH, QW> qn;
    qn.init(b);
    mm_v4f an[SLABS];
    auto fetch = [&](int c) {
        const int64_t base = ra + (int64_t)c * RCH;
        qn.load(Q + base * b, (rb - base) * b);
#pragma unroll
        for (int sl = 0; sl < SLABS; ++sl) {
            const int64_t row = base + 4 * sl + g;
            // columns in [n, round4(n)) only reach outputs that are never read
            mm_v4f v = (mm_v4f){0.f, 0.f, 0.f, 0.f};
            if (row < rb && cc < n) v = *(gc4*)(A + row * lda + cc);
            an[sl] = v;
        }
    };
    auto stage = [&](int buf) { qn.store(sQ[buf]); };
    mm_v4f acc[NB][4];
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[q][j] = (mm_v4f){0.f, 0.f, 0.f, 0.f};
    if (nch > 0) {
        fetch(0);
        stage(0);
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        mm_v4f ac[SLABS];
#pragma unroll
        for (int sl = 0; sl < SLABS; ++sl) ac[sl] = an[sl];
        if (c + 1 < nch) fetch(c + 1);
        const float* qs = sQ[c & 1];
        // A operands one slab ahead of their products (see k_gemm_nn_mfma)
        float yv[2][NB];
        auto read_slab = [&](int sl, float (&d)[NB]) {
#pragma unroll
            for (int q = 0; q < NB; ++q) d[q] = qs[(4 * sl + g) * kStageLd + 16 * q + c16];
        };
        read_slab(0, yv[0]);
#pragma unroll
        for (int sl = 0; sl < SLABS; ++sl) {
            if (sl + 1 < SLABS) read_slab(sl + 1, yv[(sl + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < NB; ++q)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[q][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(yv[sl & 1][q], ac[sl][j], acc[q][j], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (c + 1 < nch) stage((c + 1) & 1);
        __syncthreads();
    }
    // acc[q][j][r] = Z[c0 + 4 (l%16) + j][16 q + 4 (l/16) + r]
    float* out = Zp + ((int64_t)by_ * gx_ + bx_) * kTnDump + (int64_t)w * kMaxBlock * 64 + l;
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[((q * 4 + j) * 4 + r) * 64] = acc[q][j][r];
}

template <int NB, int RCH = kTnRows>
__global__ void __launch_bounds__(kThreads, 2) k_gemm_tn_mfma(const float* __restrict__ A, int64_t lda,
                                                           const float* __restrict__ Q,
                                                           float* __restrict__ Zp, int64_t m, int64_t n, int b,
                                                           int64_t rows_per_chunk) {
    k_gemm_tn_mfma_body<NB, RCH>(A, lda, Q, Zp, m, n, b, rows_per_chunk, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// Z[c][jj] = sum over the nchunk partial dumps of k_gemm_tn_mfma, in chunk
// order in FP64 (eight interleaved accumulators, added in a fixed order),
// rounded once to FP32.  One thread per dump position (ncb kTnDump of them).
__device__ __attribute__((always_inline)) inline void k_tn_sum_body(const float* __restrict__ Zp, int nchunk, int64_t per_chunk,
                                                int64_t n, int b, float* __restrict__ Z, int ldz, const int bx_, const int by_,
    const int gx_) {
    const int64_t idx = (int64_t)bx_ * blockDim.x + threadIdx.x;
    if (idx >= per_chunk) return;
    const int lane = (int)(idx & 63), r = (int)((idx >> 6) & 3);
    const int qj = (int)((idx >> 8) % (kMaxBlock / 4));
    const int64_t wq = idx / (kMaxBlock * 64);
    const int64_t c = wq * 64 + 4 * (lane & 15) + (qj & 3);
    const int jj = 16 * (qj >> 2) + 4 * (lane >> 4) + r;
    if (c >= n || jj >= b) return;
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const float* P = Zp + idx;
    int p = 0;
    for (; p + 8 <= nchunk; p += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += (double)P[(int64_t)(p + u) * per_chunk];
    }
    for (; p < nchunk; ++p) s[0] += (double)P[(int64_t)p * per_chunk];
    Z[c * ldz + jj] = (float)(((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
}

__global__ void __launch_bounds__(256) k_tn_sum(const float* __restrict__ Zp, int nchunk, int64_t per_chunk,
                                                int64_t n, int b, float* __restrict__ Z, int ldz) {
    k_tn_sum_body(Zp, nchunk, per_chunk, n, b, Z, ldz, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// Gram matrix G = Y^T Y (b x b, b <= kMaxBlock) on the FP64 matrix cores, in two
// launches.  k_gram_mfma: block p takes rows [p rpb, (p + 1) rpb) (rpb a
// multiple of 64, sized by gram_rpb so the grid covers the chip) and writes
// the upper 16 x 16 tiles (ib <= jb, row-major over the upper triangle) of
// its partial Y_p^T Y_p to Gp[p][tile][16 x 16]; the storage-type products
// are exact in FP64 and accumulate in FP64.  Rows are staged 64 at a time
// through LDS as FP64, the next stage prefetched into registers; wave w owns
// tiles w, w + 4, ....  k_gram_sum adds the partials in a fixed order and
// writes the full, exactly symmetric G.  Y row-major, or in the tiled basis
// layout when TILED.
constexpr int kGramStage = 64;
inline int64_t gram_rpb(int64_t rows) {
    const int64_t stages = (rows + kGramStage - 1) / kGramStage;
    return kGramStage * std::max<int64_t>(1, (stages + 511) / 512);
}
inline int64_t gram_parts(int64_t rows) { return std::max<int64_t>(1, (rows + gram_rpb(rows) - 1) / gram_rpb(rows)); }
// an upper bound of gram_parts(r) for every r <= rows
inline int64_t gram_parts_max(int64_t rows) { return std::max<int64_t>(1, std::min<int64_t>(512, (rows + kGramStage - 1) / kGramStage)); }
__host__ __device__ constexpr int gram_tiles(int b) { return ((b + 15) / 16) * ((b + 15) / 16 + 1) / 2; }
__device__ inline void gram_tile(int t, int nb, int* ib, int* jb) {
    int i = 0;
    while (t >= nb - i) { t -= nb - i; ++i; }
    *ib = i;
    *jb = i + t;
}

constexpr int kGramAcc = (gram_tiles(kMaxBlock) + 3) / 4;   // upper tiles per wave
template <typename T, bool TILED = false>
__device__ __attribute__((always_inline)) inline void k_gram_mfma_body(const T* __restrict__ Y, int ldy, int64_t rows, int b,
                                                        int64_t rpb, double* __restrict__ Gp, const int bx_, const int by_,
    const int gx_) {
    constexpr int PER = kGramStage * kMaxBlock / kThreads;   // staged elements per thread
    __shared__ double sY[kGramStage][kMaxBlock + 1];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nb = (b + 15) / 16, ntile = gram_tiles(b);
    int tib[kGramAcc], tjb[kGramAcc];
#pragma unroll
    for (int s = 0; s < kGramAcc; ++s) {
        const int t = w + 4 * s;
        if (t < ntile) gram_tile(t, nb, &tib[s], &tjb[s]);
        else tib[s] = tjb[s] = 0;
    }
    const int64_t ra = (int64_t)bx_ * rpb;
    const int64_t rb = min(rows, ra + rpb);
    T pre[PER];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + kThreads * q;
            const int rr = e / kMaxBlock, j = e % kMaxBlock;
            const int64_t r = r0 + rr;
            pre[q] = (r < rb && j < b) ? Y[TILED ? uvo(r, j, ldy) : r * ldy + j] : (T)0;
        }
    };
    mm_v4d acc[kGramAcc];
#pragma unroll
    for (int s = 0; s < kGramAcc; ++s) acc[s] = (mm_v4d){0.0, 0.0, 0.0, 0.0};
    fetch(ra);
    for (int64_t r0 = ra; r0 < rb; r0 += kGramStage) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + kThreads * q;
            sY[e / kMaxBlock][e % kMaxBlock] = (double)pre[q];
        }
        __syncthreads();
        if (r0 + kGramStage < rb) fetch(r0 + kGramStage);
#pragma unroll 4
        for (int kk = 0; kk < kGramStage / 4; ++kk) {
            const int rr = 4 * kk + (l >> 4);
#pragma unroll
            for (int s = 0; s < kGramAcc; ++s) {
                if (w + 4 * s < ntile)
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(sY[rr][16 * tib[s] + (l & 15)],
                                                                  sY[rr][16 * tjb[s] + (l & 15)], acc[s], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < kGramAcc; ++s) {
        const int t = w + 4 * s;
        if (t >= ntile) continue;
        double* out = Gp + ((int64_t)bx_ * ntile + t) * 256;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(4 * r + (l >> 4)) * 16 + (l & 15)] = acc[s][r];
    }
}

template <typename T, bool TILED = false>
__global__ void __launch_bounds__(kThreads) k_gram_mfma(const T* __restrict__ Y, int ldy, int64_t rows, int b,
                                                        int64_t rpb, double* __restrict__ Gp) {
    k_gram_mfma_body<T, TILED>(Y, ldy, rows, b, rpb, Gp, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// G = sum over the nparts partials of k_gram_mfma.  A block takes 32
// consecutive tile entries; thread group g (of 8) adds partials g, g + 8, ...
// in increasing order into four accumulators, and the groups' sums are added
// in group order: the result does not depend on timing.
__device__ __attribute__((always_inline)) inline void k_gram_sum_body(const double* __restrict__ Gp, int nparts, int b,
                                                  double* __restrict__ G, const int bx_, const int by_,
    const int gx_) {
    __shared__ double red[8][33];
    const int nb = (b + 15) / 16, ntile = gram_tiles(b);
    const int total = ntile * 256;
    const int o = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int e = bx_ * 32 + o;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (e < total) {
        const double* P = Gp + e;
        int p = g;
        for (; p + 24 < nparts; p += 32) {
            a0 += P[(int64_t)p * total];
            a1 += P[(int64_t)(p + 8) * total];
            a2 += P[(int64_t)(p + 16) * total];
            a3 += P[(int64_t)(p + 24) * total];
        }
        for (; p < nparts; p += 8) a0 += P[(int64_t)p * total];
    }
    red[g][o] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (g != 0 || e >= total) return;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += red[q][o];
    int ib, jb;
    gram_tile(e >> 8, nb, &ib, &jb);
    const int a = 16 * ib + ((e & 255) >> 4), c = 16 * jb + (e & 15);
    if (a >= b || c >= b || (ib == jb && a > c)) return;
    G[a * b + c] = s;
    G[c * b + a] = s;
}

__global__ void __launch_bounds__(256) k_gram_sum(const double* __restrict__ Gp, int nparts, int b,
                                                  double* __restrict__ G) {
    k_gram_sum_body(Gp, nparts, b, G, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// out[e] = sum_p P[p * stride + e] in part order; converted to Tout
template <typename Tout>
__global__ void k_sum_parts(const double* __restrict__ P, int nparts, int64_t stride, int64_t count,
                            Tout* __restrict__ out) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += P[p * stride + e];
    out[e] = (Tout)s;
}

// One block: Cholesky G = R^T R (R upper), R^{-1}; writes R (FP64, b x b)
// and R^{-1} in the storage type (b x b, row-major) for the rotation kernel.
// Rank-deficient G (a block whose columns are linearly dependent, e.g. A of
// rank below the block size): a column whose Schur-complement pivot is at
// most 4 b eps64 times its own squared norm -- below what the FP64 Gram
// resolves -- lies in the span of the columns before it and is dropped: its
// row of R and its row and column of R^{-1} are zero, so the orthonormalised
// block has a zero column there and Y = Q R still holds.  `flag` bit 0 is set
// when a column was dropped.
// Gaussian elimination of the augmented [G | I] (G = L D L^T): after step j
// every row below j has its column-j entry eliminated, so the left half ends
// as D L^T (row j = pivot d_j times row j of L^T) and the right half as
// L^{-1}.  Then R = D^{-1/2} (D L^T) and R^{-1} = L^{-T} D^{-1/2}.  The
// b x 2b augmented matrix (b <= kMaxBlock) lives in registers: thread
// (ty, tx) of a 32 x 16 grid owns rows ty + 32 p and columns tx + 16 q; step
// j publishes row j through a double-buffered LDS row, so one barrier per
// step suffices.
constexpr int kCholThreads = 512;
constexpr int kCholTY = kCholThreads / 16;   // row groups of the thread grid
template <typename T, int KB>
__device__ __attribute__((always_inline)) inline void chol_inv_fit(const double* __restrict__ G, int b,
                                                       double* __restrict__ Rout, T* __restrict__ RinvT,
                                                       int* __restrict__ flag) {
    constexpr int NP = (KB + kCholTY - 1) / kCholTY, NQ = 2 * KB / 16;
    __shared__ double s_row[2][2 * KB];
    __shared__ double s_g[KB];
    __shared__ double s_d[KB];
    __shared__ int s_drop[KB];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double g[NP][NQ];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int i = ty + kCholTY * p;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = tx + 16 * q;
            if (q < NQ / 2)
                g[p][q] = (i < b && c < b) ? G[i * b + c] : 0.0;
            else
                g[p][q] = (i < b && c - KB == i) ? 1.0 : 0.0;
        }
    }
    for (int j = threadIdx.x; j < b; j += blockDim.x) s_g[j] = G[j * b + j];
    if (ty == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) s_row[0][tx + 16 * q] = g[0][q];
    }
    __syncthreads();
    const double tol = 4.0 * b * 2.220446049250313e-16;
    for (int j = 0; j < b; ++j) {
        const double* row = s_row[j & 1];
        const double d = row[j], gjj = s_g[j];
        const bool drop = !(d > tol * gjj && gjj > 1e-300);
        const double inv_d = drop ? 0.0 : 1.0 / d;
        double rc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) rc[q] = row[tx + 16 * q];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int i = ty + kCholTY * p;
            const double f = (i > j && i < b) ? row[i] * inv_d : 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) g[p][q] -= f * rc[q];
        }
        if (threadIdx.x == 0) {
            s_d[j] = d;
            s_drop[j] = drop ? 1 : 0;
            if (drop) atomicOr(flag, 1);
        }
        const int jn = j + 1;
        if (jn < b && ty == jn % kCholTY) {
#pragma unroll
            for (int p = 0; p < NP; ++p)
                if (p == jn / kCholTY) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q) s_row[jn & 1][tx + 16 * q] = g[p][q];
                }
        }
        __syncthreads();
    }
    // R = D^{-1/2} (D L^T) (upper, dropped rows zero); R^{-1}[c][i] = L^{-1}[i][c] / sqrt(d_i)
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int i = ty + kCholTY * p;
        if (i >= b) continue;
        const double sc = s_drop[i] ? 0.0 : 1.0 / sqrt(s_d[i]);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = tx + 16 * q;
            if (q < NQ / 2) {
                if (c < b) Rout[i * b + c] = c >= i ? g[p][q] * sc : 0.0;
            } else {
                const int cc = c - KB;
                if (cc < b) RinvT[cc * b + i] = (T)(g[p][q] * sc);
            }
        }
    }
}


// The elimination in the register shape of the smallest of 32, 64, 96 and
// kMaxBlock columns that covers b: every entry of the augmented matrix takes
// the same operations in the same order in each shape, so the results are
// bitwise those of the widest one, with fewer registers and FMAs per step.
template <typename T>
__device__ __attribute__((always_inline)) inline void k_chol_inv_body(const double* __restrict__ G, int b,
                                                       double* __restrict__ Rout, T* __restrict__ RinvT,
                                                       int* __restrict__ flag, const int bx_, const int by_,
    const int gx_) {
    static_assert(kMaxBlock > 96, "widest shape");
    if (b <= 32) chol_inv_fit<T, 32>(G, b, Rout, RinvT, flag);
    else if (b <= 64) chol_inv_fit<T, 64>(G, b, Rout, RinvT, flag);
    else if (b <= 96) chol_inv_fit<T, 96>(G, b, Rout, RinvT, flag);
    else chol_inv_fit<T, kMaxBlock>(G, b, Rout, RinvT, flag);
}

template <typename T>
__global__ void __launch_bounds__(kCholThreads) k_chol_inv(const double* __restrict__ G, int b,
                                                       double* __restrict__ Rout, T* __restrict__ RinvT,
                                                       int* __restrict__ flag) {
    k_chol_inv_body<T>(G, b, Rout, RinvT, flag, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// C = A B for b x b FP64 matrices, one output per thread (grid ceil(b^2 / blockDim))
__device__ __attribute__((always_inline)) inline void k_small_gemm_body(const double* __restrict__ A, const double* __restrict__ B,
                             double* __restrict__ C, int b, const int bx_, const int by_,
    const int gx_) {
    const int e = bx_ * blockDim.x + threadIdx.x;
    if (e >= b * b) return;
    const int i = e / b, j = e % b;
    double s0 = 0.0, s1 = 0.0;
    int l = 0;
    for (; l + 1 < b; l += 2) {
        s0 += A[i * b + l] * B[l * b + j];
        s1 += A[i * b + l + 1] * B[(l + 1) * b + j];
    }
    if (l < b) s0 += A[i * b + l] * B[l * b + j];
    C[e] = s0 + s1;
}

__global__ void k_small_gemm(const double* __restrict__ A, const double* __restrict__ B,
                             double* __restrict__ C, int b) {
    k_small_gemm_body(A, B, C, b, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// out[r, 0:ldo] = in[r, 0:kin] Q[0:kin, 0:ldo]   (may run in place when ldi == ldo);
// `in` row-major, `out` row-major or, when TILED_OUT, in the tiled basis layout;
// out2 (optional) receives a second copy
template <typename T, int KC, bool TILED_OUT = false>
__device__ __attribute__((always_inline)) inline void k_rotate_plain_body(const T* in, int ldi, T* out, int ldo,
                                                           int64_t rows, int kin,
                                                           const T* __restrict__ Q, T* out2, const int bx_, const int by_,
    const int gx_) {
    constexpr int RT = KC <= 64 ? 64 : 16;
    __shared__ T sQ[KC * KC];
    __shared__ T sX[RT * KC];
    for (int e = threadIdx.x; e < kin * ldo; e += kThreads) sQ[e] = Q[e];
    const int64_t r0 = (int64_t)bx_ * RT;
    const int nr = (int)min((int64_t)RT, rows - r0);
    for (int e = threadIdx.x; e < nr * ldi; e += kThreads) sX[e] = in[r0 * ldi + e];
    __syncthreads();
    for (int e = threadIdx.x; e < nr * ldo; e += kThreads) {
        const int rr = e / ldo, j = e % ldo;
        T acc = (T)0;
        for (int c = 0; c < kin; ++c) acc += sX[rr * ldi + c] * sQ[c * ldo + j];
        const int64_t o = TILED_OUT ? uvo(r0 + rr, j, ldo) : (r0 + rr) * ldo + j;
        out[o] = acc;
        if (out2) out2[o] = acc;
    }
}

template <typename T, int KC, bool TILED_OUT = false>
__global__ void __launch_bounds__(kThreads) k_rotate_plain(const T* in, int ldi, T* out, int ldo,
                                                           int64_t rows, int kin,
                                                           const T* __restrict__ Q, T* out2 = nullptr) {
    k_rotate_plain_body<T, KC, TILED_OUT>(in, ldi, out, ldo, rows, kin, Q, out2, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// Rayleigh-Ritz core: SVD of the b x b FP64 R (row-major) by one-sided
// Jacobi in LDS, without accumulating the rotations (an order-129 matrix and
// its rotations would not fit in LDS together; eight lanes per pair).  The columns rotated
// are those of R^T (for a triangular R the one-sided Jacobi needs fewer
// sweeps on R^T than on R): W = R^T J with orthogonal columns w_j =
// sigma_j v_j, so the right vectors are v_j = w_j / sigma_j and the left ones
// u_j = R v_j / sigma_j = R w_j / sigma_j^2 (R re-read from global memory).
// Their loss of orthogonality, about the rotation threshold (b eps64) times
// sigma_1 / sigma_j, stays far below FP32 rounding for the kept triplets; a
// coarser threshold would be amplified the same way, so the FP64 one stays.
typedef WideShape RRShape;

// Column stride of the Rayleigh-Ritz matrix in LDS: for orders up to 96,
// where the Jacobi runs in a shape covering 32, 64 or 96 rows, the smallest
// stride = 4 (mod 32) doubles that covers those rows, so that pair groups
// reading different columns fall on different LDS banks; the order-129
// shape keeps its own stride.  Only addresses depend on it.
__host__ __device__ inline int rr_ldw(int N) {
    if (N > 96) return RRShape::LDW;
    const int rows = N <= 32 ? 32 : (N <= 64 ? 64 : 96);
    int st = (N + 27) / 32 * 32 + 4;
    while (st < rows) st += 32;
    return st;
}

template <typename T>
__device__ __attribute__((always_inline)) inline void k_svd_small_noj_body(
    const double* __restrict__ R, int b, int k, double* __restrict__ S, T* __restrict__ QU, T* __restrict__ QV,
    int ldo, int* __restrict__ sweeps_out, double* smem) {
    const int N = b;
    const int ldw = rr_ldw(N);
    double* W = smem;                                   // (N + 1) columns
    double* sig = W + (size_t)(N + 1) * ldw;
    double* sgn = sig + N;
    double* tmp = sgn + N;
    int* perm = (int*)(tmp + N);
    double* vmax = tmp + 2 * N;                         // per output column: signed largest entry
    // column c of W = row c of R
    for (int e = threadIdx.x; e < (N + 1) * ldw; e += blockDim.x) {
        const int col = e / ldw, row = e % ldw;
        W[e] = (row < N && col < N) ? R[col * N + row] : 0.0;
    }
    __syncthreads();
    const int sweeps = jacobi_block_fit<kMaxBlock + 1, 8>(W, N, ldw, 60);
    jacobi_sort(W, N, ldw, sig, perm, tmp);
    // sign: the largest-magnitude entry of each right vector positive
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        const double* w = W + (size_t)perm[j] * ldw;
        double best = 0.0;
        for (int e = 0; e < N; ++e)
            if (fabs(w[e]) > fabs(best)) best = w[e];
        vmax[j] = best;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += blockDim.x) sgn[j] = vmax[j] < 0.0 ? -1.0 : 1.0;
    __syncthreads();
    for (int e = threadIdx.x; e < N * ldo; e += blockDim.x) {
        const int row = e / ldo, j = e % ldo;
        double uk = 0.0, vk = 0.0;
        if (j < k) {
            const double* w = W + (size_t)perm[j] * ldw;
            const double s = sig[j];
            if (s > 0.0) {
                vk = sgn[j] * w[row] / s;
                double u = 0.0;
                for (int i = 0; i < N; ++i) u += R[row * N + i] * w[i];
                uk = sgn[j] * u / (s * s);
            }
        }
        QU[e] = (T)uk;
        QV[e] = (T)vk;
    }
    for (int j = threadIdx.x; j < k; j += blockDim.x) S[j] = sig[j];
    if (threadIdx.x == 0) *sweeps_out = sweeps;
}

template <typename T>
__global__ void __launch_bounds__(RRShape::NT) k_svd_small_noj(const double* __restrict__ R, int b, int k,
                                                              double* __restrict__ S, T* __restrict__ QU,
                                                              T* __restrict__ QV, int ldo,
                                                              int* __restrict__ sweeps_out) {
    extern __shared__ double smem[];
    k_svd_small_noj_body<T>(R, b, k, S, QU, QV, ldo, sweeps_out, smem);
}

// dynamic LDS of k_svd_small_noj for b <= kMaxBlock
__host__ __device__ constexpr size_t svd_noj_lds_doubles() {
    return (size_t)(kMaxBlock + 1) * RRShape::LDW + 6 * kMaxBlock;
}

// Start block: X[:, 0:kw] = V[:, 0:kw] (warm start), the remaining columns a
// deterministic hash in [-1, 1); identity when `ident` (b = n).  Also clears
// the four flag words of the refresh.
template <typename T>
__device__ __attribute__((always_inline)) inline void k_start_block_body(T* __restrict__ X, int ldx, int64_t n, int b, const T* __restrict__ V,
                              int ldv, int kw, uint64_t seed, int ident, int* __restrict__ flags, const int bx_, const int by_,
    const int gx_) {
    int64_t e = (int64_t)bx_ * blockDim.x + threadIdx.x;
    if (e < 4) flags[e] = 0;
    if (e >= n * b) return;
    int64_t r = e / b;
    int j = (int)(e % b);
    T v;
    if (ident) {
        v = (r == j) ? (T)1 : (T)0;
    } else if (j < kw) {
        v = V[uvo(r, j, ldv)];
    } else {
        uint64_t h = seed ^ ((uint64_t)r * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)(j + 1) * 0xC2B2AE3D27D4EB4Full);
        h ^= h >> 33; h *= 0xff51afd7ed558ccdull; h ^= h >> 33; h *= 0xc4ceb9fe1a85ec53ull; h ^= h >> 33;
        v = (T)((double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0);
    }
    X[r * ldx + j] = v;
}

template <typename T>
__global__ void k_start_block(T* __restrict__ X, int ldx, int64_t n, int b, const T* __restrict__ V,
                              int ldv, int kw, uint64_t seed, int ident, int* __restrict__ flags) {
    k_start_block_body<T>(X, ldx, n, b, V, ldv, kw, seed, ident, flags, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

template <typename Tin, typename Tout>
__global__ void k_copy2d(const Tin* __restrict__ in, int64_t ldi, Tout* __restrict__ out, int64_t ldo,
                         int64_t rows, int64_t cols) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    int64_t r = e / cols, c = e % cols;
    out[r * ldo + c] = (Tout)in[r * ldi + c];
}

constexpr int kFroRows = 16;    // rows per block of the norm / residual reductions

// ||A||_F^2 partial sums per block of kFroRows rows (FP64)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_fro2_partial(const T* __restrict__ A, int64_t lda, int64_t m,
                                                           int64_t n, double* __restrict__ part) {
    __shared__ double sred[kThreads];
    const int64_t ra = (int64_t)blockIdx.x * kFroRows;
    const int64_t rb = min(m, ra + kFroRows);
    double s = 0.0;
    for (int64_t r = ra; r < rb; ++r)
        for (int64_t c = threadIdx.x; c < n; c += kThreads) {
            double v = (double)A[r * lda + c];
            s += v * v;
        }
    sred[threadIdx.x] = s;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sred[threadIdx.x] += sred[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sred[0];
}

// E_inc^2 = ||A - U diag(S) V^T||_F^2 partial sums (eq. frob-errors), formed
// from the residual itself: grid (ceil(m/64), ceil(n/64)); a block forms its
// 64 x 64 tile of U diag(S) V^T (k-loop in LDS chunks of 16), subtracts it
// from A and sums the squares in FP64.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_resid2_partial(const T* __restrict__ A, int64_t lda,
                                                             const T* __restrict__ U, const T* __restrict__ V,
                                                             int ld, const double* __restrict__ S,
                                                             int64_t m, int64_t n, int k,
                                                             double* __restrict__ part) {
    __shared__ T sU[64][17];
    __shared__ T sV[64][17];
    __shared__ double sred[kThreads];
    const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
    const int tr = (threadIdx.x / 16) * 4, tc = (threadIdx.x % 16) * 4;
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (T)0;
    for (int l0 = 0; l0 < k; l0 += 16) {
        for (int e = threadIdx.x; e < 64 * 16; e += kThreads) {
            const int rr = e / 16, ll = e % 16;
            const int64_t r = r0 + rr, c = c0 + rr;
            const int l = l0 + ll;
            sU[rr][ll] = (r < m && l < k) ? (T)((double)U[uvo(r, l, ld)] * S[l]) : (T)0;
            sV[rr][ll] = (c < n && l < k) ? V[uvo(c, l, ld)] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int ll = 0; ll < 16; ++ll)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += sU[tr + i][ll] * sV[tc + j][ll];
        __syncthreads();
    }
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t r = r0 + tr + i, c = c0 + tc + j;
            if (r < m && c < n) {
                const double d = (double)A[r * lda + c] - (double)acc[i][j];
                s2 += d * d;
            }
        }
    sred[threadIdx.x] = s2;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sred[threadIdx.x] += sred[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = sred[0];
}

// ||G - I||_2 for a symmetric k x k G (an orthogonality residual Q^T Q - I):
// one-sided Jacobi on E = G - I; the largest column norm of the result is the
// largest |eigenvalue| of E.
__global__ void __launch_bounds__(WideShape::NT) k_sym_norm2(const double* __restrict__ G, int k,
                                                                            double* __restrict__ out,
                                                                            int* __restrict__ sweeps_out) {
    extern __shared__ double smem[];
    const int ldw = WideShape::LDW;
    // k + 1 columns: for odd k the idle pair of each round reads column k
    double* W = smem;
    double* red = W + (size_t)(k + 1) * ldw;
    for (int e = threadIdx.x; e < (k + 1) * ldw; e += blockDim.x) {
        const int col = e / ldw, row = e % ldw;
        W[e] = (row < k && col < k) ? G[row * k + col] - (row == col ? 1.0 : 0.0) : 0.0;
    }
    __syncthreads();
    const int sweeps = jacobi_block_fit<kMaxBlock + 1, WideShape::TPP>(W, k, ldw, 60);
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
        double s = 0.0;
        for (int e = 0; e < k; ++e) s += W[(size_t)c * ldw + e] * W[(size_t)c * ldw + e];
        red[c] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int c = 0; c < k; ++c) mx = fmax(mx, red[c]);
        *out = sqrt(mx);
        *sweeps_out = sweeps;
    }
}

}  // namespace isvd
