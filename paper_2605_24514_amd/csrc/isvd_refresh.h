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
#include "isvd_common.h"
#include "isvd_jacobi.h"

namespace isvd {

constexpr int kGemmRows = 64;
constexpr int kGemmK = 32;
constexpr int kChunkRows = 1024;
constexpr int kCholThreads = 1024;   // threads of the one-block Cholesky

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
// Matrix-core versions of the refresh products (b <= 96 columns).
// v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64 lane layout: A[l%16][l/16],
// B[l/16][l%16]; FP32 D[4(l/16)+r][l%16], FP64 D[4r+l/16][l%16].
typedef float mm_v4f __attribute__((ext_vector_type(4)));
typedef double mm_v4d __attribute__((ext_vector_type(4)));
constexpr int kMmK = 32;         // k-chunk staged in LDS
constexpr int kGramRows = 256;   // rows per block of the Gram partials

// Y[m x b] = A[m x n] X[n x b], FP32 in and FP32 accumulation.  A wave owns
// 32 rows (two 16-row MFMA blocks) and streams them across k on its own (no
// LDS, no block barriers): per 16-column slab, lane l loads one float4 of A
// per row block -- row l%16, columns k0 + 4 (l/16) + 0..3, 1 KB per wave
// instruction -- and the MFMA k order follows (step s takes column
// k0 + 4 (l/16) + s); X (small, cache-resident) is read in the same order
// as the B operand and shared by both row blocks.  lda % 4 == 0.  Y may be
// A itself (ldy == lda): a wave reads all of its rows before it writes them.
__global__ void __launch_bounds__(kThreads) k_gemm_nn_mfma(const float* A, int64_t lda,
                                                           const float* __restrict__ X, int ldx,
                                                           float* Y, int ldy,
                                                           int64_t m, int64_t n, int b) {
    typedef __attribute__((address_space(1))) const mm_v4f gc4;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = l >> 4, c16 = l & 15;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * 32;
    if (r0 >= m) return;
    const int nb = (b + 15) / 16;
    mm_v4f acc[2][6];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[rb][q] = (mm_v4f){0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = 0; k0 < n; k0 += 16) {
        const int64_t kc = k0 + 4 * g;
        mm_v4f a[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int64_t row = r0 + 16 * rb + c16;
            a[rb] = (mm_v4f){0.f, 0.f, 0.f, 0.f};
            if (row < m && kc < n) {
                a[rb] = *(gc4*)(A + row * lda + kc);
                // columns past n (row padding) are not part of A
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
                    if (kc + s4 >= n) a[rb][s4] = 0.f;
            }
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int64_t kk = kc + s4;
            float xv[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int j = 16 * q + c16;
                xv[q] = (q < nb && kk < n && j < b) ? X[kk * ldx + j] : 0.f;
            }
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    if (q < nb) acc[rb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][s4], xv[q], acc[rb][q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            if (q >= nb) continue;
            const int col = 16 * q + c16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + 16 * rb + 4 * g + r;
                if (row < m && col < b) Y[row * ldy + col] = acc[rb][q][r];
            }
        }
}

// Zp[chunk][c][j] = sum over the chunk's rows r of A[r][c] Q[r][j], computed
// as Z^T = Q^T A on the matrix cores (A operand Q^T, B operand A): per
// 4-row slab, lane l loads one float4 of A -- row r0 + l/16, columns
// c0 + 4 (l%16) + 0..3 (4 rows x 256 B per wave instruction) -- and feeds
// element j to the MFMA of column set j (columns c0 + 4 n + j).  A block
// covers 64 columns; its four waves take interleaved slabs of the chunk and
// are summed in a fixed order through LDS; FP32 accumulation within the
// chunk, FP64 partials out.  grid (ceil(n / 64), chunks); lda % 4 == 0.
__global__ void __launch_bounds__(kThreads) k_gemm_tn_mfma(const float* __restrict__ A, int64_t lda,
                                                           const float* __restrict__ Q, int ldq,
                                                           double* __restrict__ Zp, int64_t m, int64_t n, int b,
                                                           int64_t rows_per_chunk) {
    typedef __attribute__((address_space(1))) const mm_v4f gc4;
    __shared__ float red[64][kMaxBlock + 1];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = l >> 4, c16 = l & 15;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const int64_t ra = (int64_t)blockIdx.y * rows_per_chunk;
    const int64_t rb = min(m, ra + rows_per_chunk);
    const int nb = (b + 15) / 16;
    const int64_t cc = c0 + 4 * c16;
    mm_v4f acc[6][4];
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[q][j] = (mm_v4f){0.f, 0.f, 0.f, 0.f};
    for (int64_t s0 = ra + 4 * w; s0 < rb; s0 += 16) {
        const int64_t row = s0 + g;
        mm_v4f a = (mm_v4f){0.f, 0.f, 0.f, 0.f};
        if (row < rb && cc < n) {
            a = *(gc4*)(A + row * lda + cc);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (cc + j >= n) a[j] = 0.f;
        }
        float yv[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int jj = 16 * q + c16;
            yv[q] = (q < nb && row < rb && jj < b) ? Q[row * ldq + jj] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (q < nb) acc[q][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(yv[q], a[j], acc[q][j], 0, 0, 0);
    }
    // acc[q][j][r] = Z[c0 + 4 c16 + j][16 q + 4 g + r]; waves summed in order
    for (int ww = 0; ww < 4; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                if (q >= nb) continue;
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int jj = 16 * q + 4 * g + r;
                        float& d = red[4 * c16 + j][jj];
                        d = (ww == 0 ? 0.f : d) + acc[q][j][r];
                    }
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < 64 * b; e += kThreads) {
        const int ci = e / b, jj = e % b;
        const int64_t c = c0 + ci;
        if (c < n) Zp[((int64_t)blockIdx.y * n + c) * b + jj] = (double)red[ci][jj];
    }
}

// Gp[block] = Y[rows of block]^T Y[rows of block] (b x b) on the FP64 matrix
// cores: the storage-type products are exact in FP64 and accumulate in FP64.
// kGramRows rows per block, staged 64 at a time; wave w owns the output
// 16 x 16 blocks w, w + 4, ... of the (b/16)^2.  Y row-major, or in the
// tiled basis layout when TILED.
template <typename T, bool TILED = false>
__global__ void __launch_bounds__(kThreads) k_gram_mfma(const T* __restrict__ Y, int ldy, int64_t rows, int b,
                                                        double* __restrict__ Gp) {
    __shared__ double sY[64][kMaxBlock + 1];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nb = (b + 15) / 16, nblk = nb * nb;
    const int64_t ra = (int64_t)blockIdx.x * kGramRows;
    const int64_t rb = min(rows, ra + kGramRows);
    mm_v4d acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = (mm_v4d){0.0, 0.0, 0.0, 0.0};
    for (int64_t r0 = ra; r0 < rb; r0 += 64) {
        for (int e = threadIdx.x; e < 64 * kMaxBlock; e += kThreads) {
            const int rr = e / kMaxBlock, j = e % kMaxBlock;
            const int64_t r = r0 + rr;
            sY[rr][j] = (r < rb && j < b) ? (double)Y[TILED ? uvo(r, j, ldy) : r * ldy + j] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            const int rr = 4 * kk + (l >> 4);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int q = w + 4 * t;
                if (q < nblk) {
                    const int ib = q / nb, jb = q % nb;
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(sY[rr][16 * ib + (l & 15)], sY[rr][16 * jb + (l & 15)],
                                                                  acc[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    double* out = Gp + (int64_t)blockIdx.x * b * b;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int q = w + 4 * t;
        if (q >= nblk) continue;
        const int ib = q / nb, jb = q % nb;
        const int col = 16 * jb + (l & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * ib + 4 * r + (l >> 4);
            if (row < b && col < b) out[row * b + col] = acc[t][r];
        }
    }
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

// Gp[chunk] = Y[rows of chunk]^T Y[rows of chunk]  (b x b, FP64); Y row-major,
// or in the tiled basis layout when TILED
template <typename T, bool TILED = false>
__global__ void __launch_bounds__(kThreads) k_gram_partial(const T* __restrict__ Y, int ldy, int64_t rows,
                                                           int b, double* __restrict__ Gp) {
    __shared__ double sY[kGemmK][kMaxBlock + 1];
    const int64_t ra = (int64_t)blockIdx.x * kChunkRows;
    const int64_t rb = min(rows, ra + kChunkRows);
    const int nout = b * b;
    double acc[36];
#pragma unroll
    for (int q = 0; q < 36; ++q) acc[q] = 0.0;
    for (int64_t r0 = ra; r0 < rb; r0 += kGemmK) {
        for (int e = threadIdx.x; e < kGemmK * b; e += kThreads) {
            int rr = e / b, j = e % b;
            int64_t r = r0 + rr;
            sY[rr][j] = r < rb ? (double)Y[TILED ? uvo(r, j, ldy) : r * ldy + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 36; ++q) {
            int e = threadIdx.x + q * kThreads;
            if (e < nout) {
                int i = e / b, j = e % b;
                double s = 0.0;
                for (int rr = 0; rr < kGemmK; ++rr) s += sY[rr][i] * sY[rr][j];
                acc[q] += s;
            }
        }
        __syncthreads();
    }
    double* out = Gp + (int64_t)blockIdx.x * nout;
#pragma unroll
    for (int q = 0; q < 36; ++q) {
        int e = threadIdx.x + q * kThreads;
        if (e < nout) out[e] = acc[q];
    }
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
// Right-looking: step j takes the pivot, scales row j and updates the
// trailing upper triangle with all threads; R^{-1} row by row from the
// bottom, each step's entries in parallel.  Launched with kCholThreads.
template <typename T>
__global__ void __launch_bounds__(kCholThreads) k_chol_inv(const double* __restrict__ G, int b,
                                                       double* __restrict__ Rout, T* __restrict__ RinvT,
                                                       int* __restrict__ flag) {
    extern __shared__ double sh[];
    double* R = sh;                 // b x b row-major: the upper triangle becomes R
    double* Ri = sh + b * b;        // b x b inverse
    __shared__ int s_drop[kMaxBlock];
    __shared__ double s_dg[kMaxBlock];
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) { R[e] = G[e]; Ri[e] = 0.0; }
    __syncthreads();
    const double tol = 4.0 * b * 2.220446049250313e-16;
    // unscaled elimination (R holds the Schur complements S; row j of R is
    // S_j / sqrt(S_jj) at the end): step j reads row j and updates rows below
    // it only, so one barrier per step suffices
    for (int j = 0; j < b; ++j) {
        const double gjj = G[j * b + j];
        const double d = R[j * b + j];
        const bool drop = !(d > tol * gjj && gjj > 1e-300);
        if (threadIdx.x == 0) {
            s_drop[j] = drop ? 1 : 0;
            if (drop) atomicOr(flag, 1);
        }
        if (!drop) {
            const double inv_d = 1.0 / d;
            const int t = b - j - 1;
            for (int e = threadIdx.x; e < t * t; e += blockDim.x) {
                const int i = j + 1 + e / t, c = j + 1 + e % t;
                if (c >= i) R[i * b + c] -= R[j * b + i] * R[j * b + c] * inv_d;
            }
        }
        __syncthreads();
    }
    // scale the rows (dropped ones to zero)
    for (int j = threadIdx.x; j < b; j += blockDim.x) s_dg[j] = s_drop[j] ? 0.0 : sqrt(R[j * b + j]);
    __syncthreads();
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        const int j = e / b, c = e % b;
        if (c < j) continue;
        R[e] = s_drop[j] ? 0.0 : R[e] / s_dg[j];
    }
    __syncthreads();
    // zero the strict lower triangle (it still holds G)
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        const int i = e / b, c = e % b;
        if (i > c) R[e] = 0.0;
    }
    __syncthreads();
    // R^{-1}, rows from the bottom: Ri[i][c] = -(sum_{i<l<=c} R[i][l] Ri[l][c]) / R[i][i],
    // Ri[i][i] = 1 / R[i][i]; dropped rows and columns stay zero
    for (int i = b - 1; i >= 0; --i) {
        if (!s_drop[i]) {
            const double rii = R[i * b + i];
            for (int c = i + threadIdx.x; c < b; c += blockDim.x) {
                if (s_drop[c]) continue;
                double s0 = 0.0, s1 = 0.0;
                int l = i + 1;
                for (; l + 1 <= c; l += 2) {
                    s0 += R[i * b + l] * Ri[l * b + c];
                    s1 += R[i * b + l + 1] * Ri[(l + 1) * b + c];
                }
                if (l <= c) s0 += R[i * b + l] * Ri[l * b + c];
                Ri[i * b + c] = (c == i ? 1.0 : -(s0 + s1)) / rii;
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        Rout[e] = R[e];
        RinvT[e] = (T)Ri[e];
    }
}

// C = A B for b x b FP64 matrices (one block)
__global__ void k_small_gemm(const double* __restrict__ A, const double* __restrict__ B,
                             double* __restrict__ C, int b) {
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        int i = e / b, j = e % b;
        double s = 0.0;
        for (int l = 0; l < b; ++l) s += A[i * b + l] * B[l * b + j];
        C[e] = s;
    }
}

// out[r, 0:ldo] = in[r, 0:kin] Q[0:kin, 0:ldo]   (may run in place when ldi == ldo);
// `in` row-major, `out` row-major or, when TILED_OUT, in the tiled basis layout
template <typename T, int KC, bool TILED_OUT = false>
__global__ void __launch_bounds__(kThreads) k_rotate_plain(const T* in, int ldi, T* out, int ldo,
                                                           int64_t rows, int kin,
                                                           const T* __restrict__ Q) {
    constexpr int RT = KC <= 64 ? 64 : 16;
    __shared__ T sQ[KC * KC];
    __shared__ T sX[RT * KC];
    for (int e = threadIdx.x; e < kin * ldo; e += kThreads) sQ[e] = Q[e];
    const int64_t r0 = (int64_t)blockIdx.x * RT;
    const int nr = (int)min((int64_t)RT, rows - r0);
    for (int e = threadIdx.x; e < nr * ldi; e += kThreads) sX[e] = in[r0 * ldi + e];
    __syncthreads();
    for (int e = threadIdx.x; e < nr * ldo; e += kThreads) {
        const int rr = e / ldo, j = e % ldo;
        T acc = (T)0;
        for (int c = 0; c < kin; ++c) acc += sX[rr * ldi + c] * sQ[c * ldo + j];
        out[TILED_OUT ? uvo(r0 + rr, j, ldo) : (r0 + rr) * ldo + j] = acc;
    }
}

// Rayleigh-Ritz core: SVD of the b x b FP64 R (row-major) by the block Jacobi;
// QU = W[:, :k] (left vectors), QV = H[:, :k] (right vectors), both b x ldo in
// the storage type with zero padding; S = sigma[:k].  Dynamic LDS (2 b ldw + 6 b) doubles.
template <typename T>
__global__ void __launch_bounds__(JacobiShape<kMaxBlock + 1>::NT) k_svd_small(const double* __restrict__ R, int b, int k,
                                                        double* __restrict__ S, T* __restrict__ QU,
                                                        T* __restrict__ QV, int ldo,
                                                        int* __restrict__ sweeps_out) {
    extern __shared__ double smem[];
    const int N = b;
    const int ldw = JacobiShape<kMaxBlock + 1>::LDW;
    double* W = smem;
    double* J = W + (size_t)N * ldw;
    double* nrm = J + (size_t)N * ldw;
    double* sig = nrm + N;
    double* sgn = sig + N;
    double* tmp = sgn + N;
    int* perm = (int*)(tmp + N);
    for (int e = threadIdx.x; e < N * ldw; e += blockDim.x) {
        int col = e / ldw, row = e % ldw;
        W[e] = row < N ? R[row * N + col] : 0.0;
        J[e] = row == col ? 1.0 : 0.0;
    }
    __syncthreads();
    int sweeps = jacobi_block<kMaxBlock + 1, true>(W, J, N, ldw, 60);
    jacobi_finish(W, J, N, ldw, sig, perm, sgn, tmp);
    for (int e = threadIdx.x; e < N * ldo; e += blockDim.x) {
        int row = e / ldo, j = e % ldo;
        double uk = 0.0, vk = 0.0;
        if (j < k) {
            int c = perm[j];
            double s = sig[j];
            uk = s > 0.0 ? sgn[j] * W[(size_t)c * ldw + row] / s : 0.0;
            vk = sgn[j] * J[(size_t)c * ldw + row];
        }
        QU[e] = (T)uk;
        QV[e] = (T)vk;
    }
    for (int j = threadIdx.x; j < k; j += blockDim.x) S[j] = sig[j];
    if (threadIdx.x == 0) *sweeps_out = sweeps;
}

// FP32-storage Rayleigh-Ritz core: the same SVD of R without accumulating the
// rotations (half the LDS, so eight lanes per pair fit): W = R J with
// orthogonal columns, U_K = W diag(1/sigma), and the right vectors from
// R^T W = J diag(sigma^2), i.e. v_j = R^T w_j / sigma_j^2 (R re-read from
// global memory).  Their loss of orthogonality, about b eps64 sigma_1 / sigma_j,
// stays far below FP32 rounding for the kept triplets.
typedef JacobiShape<kMaxBlock + 1, 8> RRShape;
template <typename T>
__global__ void __launch_bounds__(RRShape::NT) k_svd_small_noj(const double* __restrict__ R, int b, int k,
                                                              double* __restrict__ S, T* __restrict__ QU,
                                                              T* __restrict__ QV, int ldo,
                                                              int* __restrict__ sweeps_out) {
    extern __shared__ double smem[];
    const int N = b;
    const int ldw = RRShape::LDW;
    double* W = smem;                                   // (N + 1) columns
    double* sig = W + (size_t)(N + 1) * ldw;
    double* sgn = sig + N;
    double* tmp = sgn + N;
    int* perm = (int*)(tmp + N);
    double* vmax = tmp + 2 * N;                         // per output column: signed largest entry
    for (int e = threadIdx.x; e < (N + 1) * ldw; e += blockDim.x) {
        const int col = e / ldw, row = e % ldw;
        W[e] = (row < N && col < N) ? R[row * N + col] : 0.0;
    }
    __syncthreads();
    const int sweeps = jacobi_block<kMaxBlock + 1, false, 8>(W, nullptr, N, ldw, 60);
    jacobi_sort(W, N, ldw, sig, perm, tmp);
    // sign: the largest-magnitude entry of each right vector positive
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        const int c = perm[j];
        const double s2 = sig[j] * sig[j];
        double best = 0.0;
        for (int e = 0; e < N; ++e) {
            double v = 0.0;
            for (int i = 0; i < N; ++i) v += R[i * N + e] * W[(size_t)c * ldw + i];
            v = s2 > 0.0 ? v / s2 : 0.0;
            if (fabs(v) > fabs(best)) best = v;
        }
        vmax[j] = best;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += blockDim.x) sgn[j] = vmax[j] < 0.0 ? -1.0 : 1.0;
    __syncthreads();
    for (int e = threadIdx.x; e < N * ldo; e += blockDim.x) {
        const int row = e / ldo, j = e % ldo;
        double uk = 0.0, vk = 0.0;
        if (j < k) {
            const int c = perm[j];
            const double s = sig[j];
            if (s > 0.0) {
                uk = sgn[j] * W[(size_t)c * ldw + row] / s;
                double v = 0.0;
                for (int i = 0; i < N; ++i) v += R[i * N + row] * W[(size_t)c * ldw + i];
                vk = sgn[j] * v / (s * s);
            }
        }
        QU[e] = (T)uk;
        QV[e] = (T)vk;
    }
    for (int j = threadIdx.x; j < k; j += blockDim.x) S[j] = sig[j];
    if (threadIdx.x == 0) *sweeps_out = sweeps;
}

// dynamic LDS of k_svd_small_noj for b <= kMaxBlock
__host__ __device__ constexpr size_t svd_noj_lds_doubles() {
    return (size_t)(kMaxBlock + 1) * RRShape::LDW + 6 * kMaxBlock;
}

// Start block: X[:, 0:kw] = V[:, 0:kw] (warm start), the remaining columns a
// deterministic hash in [-1, 1); identity when `ident` (b = n).
template <typename T>
__global__ void k_start_block(T* __restrict__ X, int ldx, int64_t n, int b, const T* __restrict__ V,
                              int ldv, int kw, uint64_t seed, int ident) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
__global__ void __launch_bounds__(JacobiShape<kMaxBlock + 1>::NT) k_sym_norm2(const double* __restrict__ G, int k,
                                                                            double* __restrict__ out,
                                                                            int* __restrict__ sweeps_out) {
    extern __shared__ double smem[];
    const int ldw = JacobiShape<kMaxBlock + 1>::LDW;
    // k + 1 columns: for odd k the idle pair of each round reads column k
    double* W = smem;
    double* red = W + (size_t)(k + 1) * ldw;
    for (int e = threadIdx.x; e < (k + 1) * ldw; e += blockDim.x) {
        const int col = e / ldw, row = e % ldw;
        W[e] = (row < k && col < k) ? G[row * k + col] - (row == col ? 1.0 : 0.0) : 0.0;
    }
    __syncthreads();
    const int sweeps = jacobi_block<kMaxBlock + 1, false>(W, nullptr, k, ldw, 60);
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
